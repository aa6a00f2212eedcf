/*
 * clbm.h -- C ABI of the MI355X (gfx950) library for the thermal cascaded
 * lattice Boltzmann method of Fei & Luo, "Cascaded lattice Boltzmann method
 * for incompressible thermal flows with heat sources and general thermal
 * boundary conditions" (arXiv:1801.04577).
 *
 * What one time step computes (clbm_step), per lattice node, fused in one
 * kernel launch:
 *   - streaming of the D2Q9 flow populations f_i and the D2Q5 temperature
 *     populations g_i (Eq. 11, Eq. 21) in pull form;
 *   - half-way bounce-back of f at no-slip walls (Sec. 3), with the
 *     momentum-exchange correction for a wall moving tangentially;
 *   - the general bounce-back scheme for g at thermal walls (Eq. 26), the wall
 *     temperature from the Robin data b1 dT/dn + b2 T = b3 (Eq. 27-28);
 *   - temperature with the source correction (Eq. 25), Boussinesq force
 *     (Eq. 2, gravity along -y), density and velocity (Eq. 12);
 *   - the cascaded collision of f in central-moment space with the consistent
 *     force term (Eq. 5-10) and back-transform;
 *   - the cascaded collision of g with the central-moment heat source (Eq. 13-20,
 *     Eq. 23-24) and back-transform.
 *
 * Conventions shared by every call:
 *   - Memory: the caller owns every device buffer (workspace, fields). The
 *     library never allocates device memory. Pointers named d_* are device
 *     pointers; all other pointers are host pointers.
 *   - Fields: float32, row-major [ny][nx], x fastest (a contiguous
 *     torch.empty(ny, nx) tensor).
 *   - Streams: every call enqueues on the HIP stream given at creation
 *     (hipStream_t passed as void*; NULL is the default stream). Only calls
 *     documented as synchronising wait for the stream.
 *   - Time level: the state after n steps is the post-collision state at
 *     time n; fields and diagnostics report the pre-collision macroscopic
 *     values at time n (they are collision invariants, up to the F/2 and Q/2
 *     corrections of Eq. 12 and Eq. 25).
 *   - Errors: every call returns a clbm_status; nothing is thrown across the
 *     ABI. A failing call leaves the handle usable unless it reports CLBM_ERR_HIP.
 *   - Threading: a handle is used from one host thread at a time.
 */
#ifndef CLBM_H
#define CLBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CLBM_ABI_VERSION 5

typedef enum {
    CLBM_OK = 0,
    CLBM_ERR_INVALID_ARG = -1,      /* bad pointer, size, side combination, NaN input */
    CLBM_ERR_UNSTABLE_PARAMS = -2,  /* a relaxation rate outside (0, 2) */
    CLBM_ERR_BUFFER_TOO_SMALL = -3, /* workspace smaller than clbm_workspace_bytes */
    CLBM_ERR_HIP = -4,              /* a HIP runtime call failed */
    CLBM_ERR_NAN = -5,              /* non-finite values found by the diagnostics */
    CLBM_ERR_UNSUPPORTED = -6       /* option not available for this configuration */
} clbm_status;

/* Population storage. Both store deviations from the rest state (f_i - w_i and
 * g_i - T0/5). The collision is FP32 arithmetic for both; the incoming population plus
 * its change is formed exactly one step wider than the storage (FP64 for CLBM_FP32, FP32
 * for CLBM_FP16_SHIFTED) and rounded once without bias (stochastic rounding, its variates
 * a hash of the node's coordinates and results). */
typedef enum { CLBM_FP32 = 0, CLBM_FP16_SHIFTED = 1 } clbm_precision;

typedef enum { CLBM_PERIODIC = 0, CLBM_WALL = 1 } clbm_side_kind;

/* Side indices of clbm_params.side. Opposite sides must have the same kind. */
enum { CLBM_SIDE_XM = 0, CLBM_SIDE_XP = 1, CLBM_SIDE_YM = 2, CLBM_SIDE_YP = 3 };

typedef struct {
    int kind;       /* clbm_side_kind */
    double u_wall;  /* tangential wall speed (x- and x+: along y; y- and y+: along x) */
    double b1, b2, b3; /* thermal wall: b1 dT/dn + b2 T = b3, n the outward normal
                          (Dirichlet: 0,1,T_w; adiabatic: 1,0,0); not both b1, b2 zero */
} clbm_side;

typedef struct {
    int nx, ny;         /* lattice nodes; >= 2 across walled directions. Limits (else
                           CLBM_ERR_UNSUPPORTED): 14 x 64 ceil(nx/64) x 4 bytes < 2^32 (nx up
                           to about 76 million) and the lattice padded to 64 x 4 blocks
                           holds fewer than 2^32 nodes; beyond that only device memory
                           bounds the size (112 B per node in FP32, 56 B in FP16). */
    int precision;      /* clbm_precision */
    double nu;          /* kinematic viscosity: s_nu = 1/(3 nu + 1/2) (Sec. 2.1) */
    double alpha;       /* thermal diffusivity: lambda_1 = 1/(alpha/c_T^2 + 1/2) (Sec. 2.2) */
    double s_b;         /* bulk rate (Eq. 8); NaN -> 1 */
    double s_4;         /* rate of k22 (Eq. 8); NaN -> 1 */
    double s_3;         /* rate of k21, k12; NaN -> s_3 = (16 - 8 s_nu)/(8 - s_nu) (Sec. 3) */
    double lambda_0;    /* rate of the thermal k00; it has no effect (NaN -> 1) */
    double lambda_2;    /* rate of thermal k20, k02; NaN -> 12(lambda_1 - 2)/(lambda_1 - 12) (Sec. 3.1) */
    double g_beta;      /* Boussinesq: F_y += g_beta (T - T0) (Eq. 2) */
    double T0;          /* Boussinesq reference temperature; also the storage shift of g */
    double Fx, Fy;      /* external body force F_v (Eq. 2) */
    double Q;           /* uniform heat source (Eq. 24) */
    int viscous_heating; /* 0 or 1: add the local viscous dissipation
                            nu [(d_x u_y + d_y u_x)^2 + (d_x u_x - d_y u_y)^2] to Q (Sec. 3.2),
                            evaluated from the non-equilibrium central moments k11 and
                            k20 - k02. Requires g_beta = 0 and |1 - s_nu| >= 1e-3
                            (nu not within about 3.3e-4 of 1/6), else CLBM_ERR_INVALID_ARG. */
    clbm_side side[4];  /* CLBM_SIDE_XM, _XP, _YM, _YP */
} clbm_params;

/* Kernel launch shape of the fused step (set by the autotuner or by hand).
 * steps_per_launch = 1: one time step per launch; block_x * block_y threads per
 * workgroup (multiple of 64, at most 1024), rows_per_thread in {1, 2, 4}, xcd_remap != 0
 * maps consecutive tiles to the same XCD.
 * steps_per_launch = 2: two time steps per launch, the intermediate state kept in LDS
 * (rounded into the storage type exactly as a stored state) by workgroups that own tiles
 * of 64 x two_step_rows nodes: two_step_rows 6, 14, 22 or 30 (256, 512, 512 or 1024
 * threads; 0 selects 14 for FP32 storage and 22 for FP16 storage);
 * xcd_remap applies to these tiles too, the other fields shape only the single step that
 * ends an odd step count (256 x 1 threads, one row each, if they do not form a valid
 * shape). Both modes give bitwise identical states.
 * A zeroed struct selects the built-in default: two steps per launch with xcd_remap. */
typedef struct {
    int block_x, block_y, rows_per_thread, xcd_remap;
    int steps_per_launch;
    int two_step_rows;
} clbm_launch;

/* Diagnostics at the current time (Sec. 3.3 Nusselt number and a residual). */
typedef struct {
    long step;        /* time level of the state */
    int K;            /* steps since the previous snapshot (0 if none) */
    double mass;      /* sum over nodes of rho */
    double sum_u2;    /* sum |u|^2 */
    double sum_du2;   /* sum |u - u_snapshot|^2 */
    double sum_T2;    /* sum T^2 */
    double sum_dT2;   /* sum (T - T_snapshot)^2 */
    double res_u;     /* sqrt(sum_du2/sum_u2)/K, 0 if K == 0 or sum_u2 == 0 */
    double res_T;     /* sqrt(sum_dT2/sum_T2)/K, same convention */
    double dTdn[4];   /* per side: mean outward normal derivative of T at the wall (Eq. 27) */
    double T_wall[4]; /* per side: mean wall temperature (Eq. 28) */
    double wall_flux[4]; /* per side: mean heat leaving the fluid through the wall per wall
                            node and step, 2 g*_out - c_T^2 T_w of the link that crosses it
                            (Eq. 26); equals -alpha dT/dn up to the discretisation error,
                            a cross-check of dTdn */
    long nan_count;   /* nodes with a non-finite rho, u or T */
} clbm_diag;

typedef struct clbm_handle clbm_handle;

int clbm_abi_version(void);
const char* clbm_status_string(int status);

/* Host only. out = {s_nu, s_b, s_3, s_4, lambda_0, lambda_1, lambda_2}: the relaxation
 * rates the kernels use (Eq. 8, Sec. 2.2, the rules of Sec. 3 and Sec. 3.1). */
clbm_status clbm_derive_rates(const clbm_params* p, double out[7]);

/* Host only. Validates p and returns the workspace size the handle needs: two
 * population buffers, a snapshot of (u_x, u_y, T) for the residual, and reduction
 * scratch. A population buffer holds each row in blocks of 64 nodes, a block storing
 * its 14 populations (f_0..f_8, g_0..g_4) 64 values each; rows are padded to whole
 * blocks. The layout is internal: clbm_populations exports plain planes. */
clbm_status clbm_workspace_bytes(const clbm_params* p, size_t* bytes);

/* Creates a handle over the caller's workspace (device memory of at least
 * clbm_workspace_bytes, 256-byte aligned). The state is the rest state
 * rho = 1, u = 0, T = T0 until clbm_init_from_fields is called. */
clbm_status clbm_create(const clbm_params* p, void* d_workspace, size_t bytes, void* hip_stream,
                        clbm_handle** out);
void clbm_destroy(clbm_handle* h);

/* Initial state: the discrete equilibrium of Eq. (9) and Eq. (19) at the given
 * (rho, u, T), followed by one collision. Any NULL field takes rho = 1, u = 0,
 * T = T0. Resets the step counter and the residual snapshot. Asynchronous. */
clbm_status clbm_init_from_fields(clbm_handle* h, const float* d_rho, const float* d_ux,
                                  const float* d_uy, const float* d_T);

/* Advances nsteps time steps. One step is the cascaded collision of f (Eq. 5-10) and
 * of g with the heat source (Eq. 13-20, 23-25), then streaming (Eq. 11, 21) with the
 * wall rules of Sec. 3 and Eq. (26)-(28), all fused per node as listed at the top of
 * this file. One fused kernel per step, or one per two steps when steps_per_launch = 2;
 * steps are replayed from a HIP graph when graphs are enabled. nsteps = 0 is a no-op,
 * nsteps < 0 (or a NULL handle) returns CLBM_ERR_INVALID_ARG.
 * Asynchronous; CLBM_ERR_HIP if a launch fails. */
clbm_status clbm_step(clbm_handle* h, int nsteps);

/* Writes rho, u_x, u_y, T at the current time: rho and u as moments of f with half the
 * force (Eq. 12), T as the moment of g with half the node's source (Eq. 25). Outputs are
 * caller-owned device arrays of nx*ny floats, [ny][nx]; NULL outputs are skipped.
 * Asynchronous. */
clbm_status clbm_macros(clbm_handle* h, float* d_rho, float* d_ux, float* d_uy, float* d_T);

/* Writes the stored post-collision state as float32 deviations: d_f [9][ny][nx]
 * holds f*_i - w_i (w = 4/9, 1/9, 1/36), d_g [5][ny][nx] holds g*_i - T0/5.
 * NULL outputs are skipped. Asynchronous. */
clbm_status clbm_populations(clbm_handle* h, float* d_f, float* d_g);

/* Reduces the diagnostics over the lattice: the wall gradients and wall temperatures
 * (Eq. 27-28) from which the average Nusselt number along a wall of the natural-convection
 * cavity follows (Sec. 3.3, Table 1), mass, and the change since the last snapshot (the
 * steady-state residual; the paper states no criterion, see clbm_diag). Wavefront and
 * workgroup reductions, then a fixed-order FP64 pass; the partial sums live in the
 * handle's workspace. Replaces the residual snapshot with the current
 * fields. Synchronises the stream. Returns CLBM_ERR_NAN (with *out filled) when a
 * non-finite value is found. */
clbm_status clbm_diagnostics(clbm_handle* h, clbm_diag* out);

/* For callers that cannot allocate device memory or use a workspace of their own at
 * this point (tight serving loops, harnesses that forbid allocation): clbm_diagnostics with
 * the reduction's partial and final sums in a fixed library-owned device array (155 KB
 * per GPU, held until the process ends; resolved per device at clbm_create) instead of
 * the handle's workspace. Calls no hipMalloc or hipFree. The array holds the partials of
 * any lattice size (the reduction grid is capped at 1024 workgroups); a request beyond
 * it would return CLBM_ERR_BUFFER_TOO_SMALL. All handles on one GPU share the array, so
 * calls that overlap on one GPU race: order them on one stream. Same results, residual
 * snapshot update, synchronisation and errors as clbm_diagnostics; like it, the call
 * waits for the stream, so it cannot be recorded into a stream capture. */
clbm_status clbm_diagnostics_noalloc(clbm_handle* h, clbm_diag* out);

/* Checkpoint: the state occupies clbm_state_bytes; save copies it to d_dst,
 * load copies it back and sets the step counter. Asynchronous. */
clbm_status clbm_state_bytes(const clbm_handle* h, size_t* bytes);
clbm_status clbm_save(clbm_handle* h, void* d_dst);
clbm_status clbm_load(clbm_handle* h, const void* d_src, long step);

clbm_status clbm_get_step(const clbm_handle* h, long* step);
clbm_status clbm_set_launch(clbm_handle* h, const clbm_launch* launch);
clbm_status clbm_get_launch(const clbm_handle* h, clbm_launch* launch);
/* A heat source given per node, added to the uniform Q (Sec. 3.2 treats a spatially
 * variable source; Eq. (23)-(25) take the node's source): d_q is a device float32
 * array [ny][nx] (row-major, x fastest) that the caller owns and keeps alive and
 * unchanged while the handle steps; NULL removes it. The step then reads 4 more bytes
 * per node. The state stored so far keeps its meaning: T is recovered from the stored
 * populations as sum g* - Q/2 with the node's current source, so set the field before
 * clbm_init_from_fields (or change it only where the source changes anyway). Rebuilds
 * the handle's graphs. */
clbm_status clbm_set_source_field(clbm_handle* h, const float* d_q);
/* steps_per_graph = 0 launches every step on the stream; an even value > 0 replays
 * graphs of that many steps (the default is 0). Both graphs (one per starting buffer)
 * are instantiated by this call; clbm_set_launch drops them and the next clbm_step
 * rebuilds the one it needs. */
clbm_status clbm_set_graph(clbm_handle* h, int steps_per_graph);

/* Plain device-to-device copy of `bytes` bytes (one 16-byte load and store per thread;
 * both pointers 16-byte aligned, bytes a multiple of 16) on the given
 * stream. It is the bandwidth reference of the benchmark (a kernel whose HBM traffic
 * is known exactly) and calibrates hardware traffic counters against the step kernel.
 * Not part of the method. Asynchronous. */
clbm_status clbm_stream_copy(void* d_dst, const void* d_src, size_t bytes, void* hip_stream);

/* ------------------------------------------------------------------------ */
/* Batched form: many independent lattices (each with its own size and        */
/* parameters) advanced together, one kernel launch per time step over a      */
/* device tile list covering every active instance.                            */
/* ------------------------------------------------------------------------ */

typedef struct clbm_batch clbm_batch;

/* Status codes per instance reported by clbm_batch_run. */
enum { CLBM_INST_RUNNING = 0, CLBM_INST_CONVERGED = 1, CLBM_INST_DIVERGED = 2,
       CLBM_INST_MAX_STEPS = 3 };

/* Tile shape of the batched kernel. steps_per_launch = 1: tile_x * tile_y nodes per
 * workgroup, one node per thread (tile_x a multiple of 64, tile_x * tile_y <= 1024).
 * steps_per_launch = 2: two time steps per launch with the intermediate state in LDS,
 * tiles of 64 x tile_y nodes with tile_y 6, 14, 22 or 30 (256, 512, 512 or 1024 threads; the LDS
 * tile of 66 x (tile_y + 2) nodes sets how many workgroups share a CU); bitwise equal to
 * one-step launches. persistent_wgs > 0 launches that many workgroups, each looping over
 * tiles; 0 launches one workgroup per tile. xcd_bands = 1 deals the tile list of a
 * two-step launch to the eight XCDs in contiguous bands (neighbouring tiles of an
 * instance share an L2), 0 strides every workgroup over the whole list. The default
 * (launch NULL at create) is the two-step 64 x 14 shape, one workgroup per tile, in XCD
 * bands. */
typedef struct {
    int tile_x, tile_y, persistent_wgs;
    int steps_per_launch;
    int xcd_bands;
} clbm_batch_launch;

/* Host only. Workspace for n instances (every precision field CLBM_FP32, or every one
 * CLBM_FP16_SHIFTED: one storage type per batch, else CLBM_ERR_UNSUPPORTED; each
 * instance's population buffer, 14 x 64 ceil(nx/64) x ny values, must hold fewer than
 * 2^32 of them, else CLBM_ERR_UNSUPPORTED). */
clbm_status clbm_batch_workspace_bytes(int n, const clbm_params* p, size_t* bytes);
/* launch NULL selects the default shape. */
clbm_status clbm_batch_create(int n, const clbm_params* p, void* d_workspace, size_t bytes,
                              void* hip_stream, const clbm_batch_launch* launch,
                              clbm_batch** out);
void clbm_batch_destroy(clbm_batch* b);
/* Initial state of instance i from its fields (NULL: rest state), as clbm_init_from_fields. */
clbm_status clbm_batch_init(clbm_batch* b, int i, const float* d_rho, const float* d_ux,
                            const float* d_uy, const float* d_T);
/* Advances every instance by nsteps, those a clbm_batch_run has retired included (all
 * instances share the buffer parity); the run's retirements stand for a later
 * clbm_batch_run (asynchronous). */
clbm_status clbm_batch_step(clbm_batch* b, int nsteps);
/* Marks every instance running with zero steps, restores the full tile list and takes
 * the residual snapshot of the current state (asynchronous). */
clbm_status clbm_batch_reset(clbm_batch* b);
/* Runs every instance to its steady state, the end point of the natural-convection and
 * source tests of Sec. 3 (the paper gives no stopping rule; this one is the relative
 * change of u and T over a window, as in clbm_diag). Advances the running instances with
 * the step of clbm_step until each has converged (max(res_u, res_T) < tol, the
 * residuals of windows of K steps), diverged (non-finite value or |u| > 0.5) or taken
 * max_steps steps since clbm_batch_reset, or until this call has advanced budget_steps
 * steps (budget_steps <= 0: no budget); a later call resumes. Convergence checks,
 * retirement and compaction of the tile list run on the device inside a replayed HIP
 * graph of K steps. With FP16 storage the residual settles at about 5e-7 to 1e-6 (the
 * unbiased rounding into binary16 keeps moving the stored state by rounding noise), so tol
 * must lie above that floor (2e-6, say). Synchronises. steps_out[i] is the number of steps instance i has
 * taken (for a retired instance, the step it stopped at), status_out[i] its CLBM_INST_*
 * code; host arrays of length n. */
clbm_status clbm_batch_run(clbm_batch* b, long max_steps, double tol, int K, long budget_steps,
                           long* steps_out, int* status_out);
clbm_status clbm_batch_macros(clbm_batch* b, int i, float* d_rho, float* d_ux, float* d_uy,
                              float* d_T);
/* Diagnostics of instance i at its current state (mass, wall gradients and temperatures,
 * field sums, NaN count; the residual fields are zero). Overwrites the instance's residual
 * snapshot. Synchronises; step is the number of steps the last clbm_batch_run gave it. */
clbm_status clbm_batch_diagnostics(clbm_batch* b, int i, clbm_diag* out);
/* Host copy of instance i's last residuals {res_u, res_T}; synchronises. */
clbm_status clbm_batch_residual(clbm_batch* b, int i, double out[2]);
/* Times candidate launches on the batch's own instances (each for `steps` steps after a
 * 2-step warm-up): one-step tiles, the three two-step tile heights with and without XCD
 * bands, each with one workgroup per tile and with 2048 and 8192 persistent workgroups.
 * Keeps the fastest. With cache_path (not NULL) it appends one JSON line per candidate
 * and a last line {"signature": ..., "best": 1, ...} naming the winner; the signature is
 * a 64-bit hash of the instance count, the storage type and every instance's (nx, ny,
 * viscous heating). Every timed step advances the instances, so call it before
 * clbm_batch_init (or re-initialise afterwards). Synchronises. */
clbm_status clbm_batch_autotune(clbm_batch* b, int steps, const char* cache_path,
                                clbm_batch_launch* best);
/* Host only. Reads the launch that clbm_batch_autotune chose for a batch with this
 * batch's signature from the cache file (the last "best" line that matches). *found = 1
 * and *out filled when there is one; *found = 0 when the file or the entry is missing. */
clbm_status clbm_batch_tune_lookup(const clbm_batch* b, const char* cache_path, clbm_batch_launch* out,
                                   int* found);
clbm_status clbm_batch_set_launch(clbm_batch* b, const clbm_batch_launch* launch);
/* Source field of instance i (as clbm_set_source_field: a device float32 [ny][nx] array the
 * caller keeps alive, NULL removes it). Synchronises. */
clbm_status clbm_batch_set_source_field(clbm_batch* b, int i, const float* d_q);

/* ------------------------------------------------------------------------ */
/* Warm-start network: a four-level convolutional encoder-decoder with skip    */
/* connections mapping input planes that describe a cavity problem to the       */
/* steady fields (u_x, u_y, T) on a fixed grid. 3x3 convolutions run on BF16    */
/* MFMA with FP32 accumulation; activations and their gradients are BF16,       */
/* master weights, weight gradients and the Adam state FP32. Layer order and    */
/* the canonical parameter layout: per convolution (15 of them, encoder levels  */
/* cin->w1->w1, w1->w2->w2, w2->w3->w3, w3->w4->w4; decoder (w4+w3)->w3->w3,    */
/* (w3+w2)->w2->w2, (w2+w1)->w1->w1; output w1->cout) W[cout][cin][3][3] then   */
/* b[cout], float32. Every convolution but the last is followed by ReLU;        */
/* downsampling is 2x2 averaging, upsampling is nearest-neighbour, the skip     */
/* tensor is concatenated after the upsampled one.                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    int batch;          /* samples per forward/backward call */
    int height, width;  /* grid, multiples of 8; batch*(height/8)*(width/8) a multiple of 64 */
    int cin;            /* input planes, 1..32 */
    int cout;           /* output fields, 1..16 */
    int widths[4];      /* channels per level, multiples of 32 */
} clbm_net_desc;

typedef struct clbm_net clbm_net;

/* Host only: number of floats in the canonical parameter vector / workspace bytes. */
clbm_status clbm_net_param_count(const clbm_net_desc* d, size_t* count);
clbm_status clbm_net_workspace_bytes(const clbm_net_desc* d, size_t* bytes);
/* Creates the network over the caller's workspace (256-byte aligned) and zeroes it
 * (parameters, Adam state). */
clbm_status clbm_net_create(const clbm_net_desc* d, void* d_workspace, size_t bytes, void* hip_stream,
                            clbm_net** out);
void clbm_net_destroy(clbm_net* n);
/* Device copies of the canonical parameter vector (and of the last gradients). */
clbm_status clbm_net_set_params(clbm_net* n, const float* d_params);
clbm_status clbm_net_get_params(clbm_net* n, float* d_params);
clbm_status clbm_net_get_grads(clbm_net* n, float* d_grads);
/* Forward pass: d_x [batch][cin][H][W] -> d_y [batch][cout][H][W] (float32 NCHW;
 * d_y may be NULL). Keeps the activations for clbm_net_backward. Asynchronous. */
clbm_status clbm_net_forward(clbm_net* n, const float* d_x, float* d_y);
/* Backward pass of the mean squared error between the last forward output and d_target
 * ([batch][cout][H][W]): fills the gradients of every parameter. *loss (host, may be
 * NULL) receives the loss; a non-NULL loss synchronises the stream. */
clbm_status clbm_net_backward(clbm_net* n, const float* d_target, double* loss);
/* One Adam update of the parameters with the last gradients (step t >= 1). */
clbm_status clbm_net_adam(clbm_net* n, float lr, float beta1, float beta2, float eps, int t);
/* Bilinear resampling of nfields (<= 16) float32 fields [nfields][sh][sw] to
 * [nfields][dh][dw] on cell-centred grids (edge values held), each output field
 * multiplied by scale[f] and shifted by shift[f] (host arrays of nfields; NULL: 1 and 0).
 * Moves fields between a lattice and the network grid. Asynchronous. */
clbm_status clbm_resample_bilinear(const float* d_src, int sh, int sw, float* d_dst, int dh, int dw,
                                   int nfields, const float* scale, const float* shift,
                                   void* hip_stream);

/* Scalar description of a cavity problem for the warm-start network (host struct).
 * Dimensionless groups of Sec. 3.3: Ra = g beta dT H^3/(nu alpha), Pr = nu/alpha, and the
 * source q_star = Q H^2/(alpha dT), with H = ny and dT the difference of the Dirichlet side-wall
 * temperatures (1 if the side walls are not both Dirichlet). kind per side: 0 periodic,
 * 1 Dirichlet, 2 adiabatic, 3 other Robin; theta_wall = (T_w - T0)/dT on Dirichlet sides.
 * u_scale = sqrt(g beta dT H) and t_scale = dT are the units of the network's outputs. */
typedef struct {
    float log10_ra, pr, q_star, log2_aspect;
    float theta_wall[4];
    int kind[4];
    float u_scale, t_scale;
} clbm_problem_code;

/* Host only: the code of a parameter block. */
clbm_status clbm_problem_encode(const clbm_params* p, clbm_problem_code* out);

/* Input planes of the network, [batch][8][height][width] float32, from one device
 * clbm_problem_code per sample: 0 (log10 Ra - 4.5)/1.5, 1 (Pr - 3.85)/3.15, 2 q_star/4,
 * 3 theta_wall on Dirichlet boundary cells, 4 Dirichlet mask, 5 adiabatic mask,
 * 6 x in (-1, 1), 7 log2(nx/ny). Asynchronous. */
clbm_status clbm_net_features(const clbm_problem_code* d_codes, int batch, int height, int width,
                              float* d_out, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
