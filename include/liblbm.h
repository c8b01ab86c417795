/*
 * liblbm -- single-relaxation-time Shan-Chen D3Q19 lattice Boltzmann on
 * AMD Instinct MI355X (gfx950).
 *
 * The method is that of Chiappini, Xue, Falcucci & Sbragaglia, "Ligament
 * break-up simulation through pseudo-potential Lattice Boltzmann Method",
 * Section 2: D3Q19 populations on a periodic Cartesian grid, BGK relaxation
 * with one time tau (Eqs. 1 and 3), the second-order equilibrium (Eq. 2,
 * with its leading 1), moments (Eq. 4), the single-belt pseudo-potential
 * force (Eq. 5) with psi = rho0 (1 - exp(-rho/rho0)), entering through the
 * velocity shift u' = u + tau F / rho of Eq. (6).  Lattice units: dt = dx = 1,
 * c_s^2 = 1/3.  The extra forcing term F_a of Eq. (3) is zero: the
 * interaction acts only through the shift.
 *
 * Conventions shared by every call
 *   - Grid nx * ny * nz, periodic in all three directions, each extent >= 1.
 *     Node index ((z * ny) + y) * nx + x, x fastest.
 *   - Canonical population order (used by every FP64 export/import):
 *       0 rest; 1..6 = +x, -x, +y, -y, +z, -z;
 *       7..18 = +x+y, -x-y, +x-y, -x+y, +x+z, -x-z, +x-z, -x+z,
 *               +y+z, -y-z, +y-z, -y+z   (opposite directions adjacent).
 *     A population array is [19][n] doubles, population-major.
 *     "State at step t" means f_a(x, t): post-streaming, before collision.
 *   - G is signed; phase separation needs G < 0 (the paper's G0 = 5.3 of
 *     Section 4 is G = -5.3 here).
 *   - Every call returns an lbm_status (0 = LBM_OK).  No call throws or
 *     aborts.  On error the thread-local message lbm_last_error() says why,
 *     and state is left as it was, except after LBM_ERR_DEVICE, which
 *     poisons the context (later calls on it return LBM_ERR_STATE).
 *   - Device memory is owned by the caller: the library allocates none for
 *     the lattice, only borrows the workspace given to lbm_create.
 *   - Work is ordered on the HIP stream given at creation.  Only calls that
 *     return host data synchronise that stream (lbm_diagnostics,
 *     lbm_read_diag_history, lbm_get_fields with on_device = 0,
 *     lbm_coexistence, lbm_autotune).
 */
#ifndef LIBLBM_H
#define LIBLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_ERR_INVALID_ARG = -1,    /* bad argument; nothing changed */
    LBM_ERR_UNSUPPORTED = -2,    /* valid request the library does not provide */
    LBM_ERR_DEVICE = -3,         /* a HIP call failed; the context is poisoned */
    LBM_ERR_STATE = -4,          /* call on a poisoned or uninitialised object */
    LBM_ERR_DIVERGED = -5,       /* non-finite or non-positive density found */
    LBM_ERR_BUFFER_TOO_SMALL = -6
} lbm_status;

/* Pseudo-potential form (Section 2, below Eq. 5): psi = rho0 (1 - exp(-rho/rho0)). */
typedef enum { LBM_PSI_EXP = 0 } lbm_psi;

/*
 * Population storage.  F64 and F32 store f_a as is and compute in the same
 * precision (152 and 76 bytes per node).  F16S and BF16S store the shifted
 * value f_a - w_a rho_ref of all 19 populations in IEEE half / bfloat16
 * (round-to-nearest-even both ways) and compute in FP32 (38 bytes per node).
 * F16M and BF16M store the 18 moving populations the same way and the rest
 * population, shifted, in FP32 (40 bytes per node); the arithmetic is FP32
 * on the shifted values, and each collision sets the rest population to the
 * node's mass minus the moving populations as they are stored, so the
 * stored mass of a node equals the mass the collision conserves (Eq. 4) to
 * FP32 rounding instead of moving by 19 half-precision roundings per step.
 * The FP32-rest kinds run the BGK collision on the run-time tiles
 * (tile_x = 0) only.
 */
typedef enum {
    LBM_F64 = 0, LBM_F32 = 1, LBM_F16S = 2, LBM_BF16S = 3, LBM_F16M = 4, LBM_BF16M = 5
} lbm_storage;

typedef struct {
    int32_t nx, ny, nz; /* grid extents, each >= 1; 19 nx ny and n = nx ny nz <= 2^31 - 1 */
    double tau;         /* relaxation time, > 0.5 (Eq. 1) */
    double G;           /* interaction strength of Eq. (5), signed, finite */
    int32_t psi;        /* lbm_psi */
    double rho0;        /* reference density of psi, > 0 (the paper uses 1) */
    int32_t storage;    /* lbm_storage */
    double rho_ref;     /* shift density for F16S/BF16S (ignored otherwise) */
} lbm_params;

typedef struct lbm_ctx lbm_ctx;

/*
 * Bytes of device workspace a context with these parameters needs (two
 * lattices of 19 populations plus diagnostic buffers), or 0 if the
 * parameters are invalid.
 */
size_t lbm_workspace_bytes(const lbm_params *p);

/*
 * Create a context.  d_workspace: device pointer, 256-byte aligned, at least
 * lbm_workspace_bytes(p) bytes, owned by the caller and borrowed until
 * lbm_destroy.  hip_stream: a hipStream_t (NULL = the null stream).  The
 * lattice content is undefined until lbm_init_ligament or
 * lbm_set_populations.  Errors: INVALID_ARG (bad params, null pointers,
 * misalignment), BUFFER_TOO_SMALL, DEVICE.
 */
int lbm_create(const lbm_params *p, void *d_workspace, size_t ws_bytes, void *hip_stream,
               lbm_ctx **out);

/* Release host-side state and captured graphs (after waiting for the stream
 * when a captured graph exists).  Never frees the workspace. */
int lbm_destroy(lbm_ctx *ctx);

/*
 * Coexisting liquid/vapour densities for (G, tau, psi, rho0), in FP64 on the
 * current HIP device.  A flat interface on a 1 x 1 x 128 periodic slab
 * (liquid on [32, 96), tanh start of width 4 between the densities of
 * lbm_equal_area, at rest) is advanced in chunks of 1000 steps of the same
 * update (Eqs. 2-6).  For tau < 1 it is first relaxed at tau = 1 and at tau
 * lowered in steps of 0.05 (each stage until the largest density change over
 * a chunk is below 1e-8, at most 100 chunks), because a direct low-tau start
 * can blow up in its initial transient.  At the requested tau it runs until
 * the chunk change is below 1e-12, until that change has grown 100-fold
 * above its smallest value once the smallest is below 1e-8, or for 200
 * chunks; the densities at z = 64 (liquid) and z = 0 (vapour) of the chunk
 * with the smallest change are returned.  With the velocity-shift forcing
 * they depend on tau as well as G.  Synchronous.  Errors: INVALID_ARG
 * (G >= -4/rho0 has no coexistence, tau <= 0.5, null outputs), DIVERGED,
 * DEVICE.
 */
int lbm_coexistence(double G, double tau, int32_t psi, double rho0, double *rho_l,
                    double *rho_v);

/*
 * Multiple-relaxation-time (MRT) collision, the operator the paper's
 * conclusion names as future work (it lets the viscosity change at a fixed
 * density ratio; the paper gives no details).  Moment basis of d'Humieres,
 * Ginzburg, Krafczyk, Lallemand and Luo (Phil. Trans. R. Soc. A 360, 2002)
 * for D3Q19: rho, e, eps, j, q, 3p_xx, 3pi_xx, p_ww, pi_ww, p_xy, p_yz, p_xz,
 * m.  Equilibrium moments: those of the second-order equilibrium of Eq. (2),
 * so that all rates equal to 1/tau give BGK.  The viscous moments (p_xx,
 * p_ww, p_xy, p_yz, p_xz) relax at 1/tau: nu = (tau - 1/2)/3 as for BGK;
 * the bulk viscosity is (2/9)(1/s_e - 1/2).  The force enters as the
 * velocity shift of Eq. (6) in moment space: the equilibrium is taken at
 * momentum j + F / s_j.  Every rate lies in (0, 2); s_j <= 0 selects
 * s_j = 1/tau (the BGK shift u + tau F / rho).  d'Humieres et al. suggest
 * s_e = 1.19, s_eps = s_pi = 1.4, s_q = 1.2, s_m = 1.98.
 */
typedef struct {
    double s_e, s_eps, s_q, s_pi, s_m, s_j;
} lbm_mrt;

/*
 * lbm_coexistence with the MRT collision at these rates (the tau stages
 * change only the viscous rate).  Errors as lbm_coexistence; INVALID_ARG for
 * rates outside (0, 2).
 */
int lbm_coexistence_mrt(double G, double tau, const lbm_mrt *mrt, int32_t psi, double rho0,
                        double *rho_l, double *rho_v);

/*
 * lbm_coexistence for m (G, tau) pairs at once: the m flat-interface runs
 * (each as described for lbm_coexistence, with the same stages and stopping
 * rule, hence the same densities) advance together, one workgroup each, so m
 * runs take about as long as the slowest one.  mrt: NULL for BGK, else the
 * MRT rates shared by all runs.  Outputs are host arrays of m entries:
 * status[j] is LBM_OK or LBM_ERR_DIVERGED, and a diverged run's densities
 * are NaN.  Returns LBM_OK if every run converged, LBM_ERR_DIVERGED if any
 * diverged (the others' results are valid).  Synchronous.  Errors before any
 * device work: INVALID_ARG (m < 1, a NULL array, any case's G or tau invalid
 * as for lbm_coexistence; the message names the case), UNSUPPORTED (psi);
 * then DEVICE.
 */
int lbm_coexistence_many(int32_t m, const double *G, const double *tau, const lbm_mrt *mrt,
                         int32_t psi, double rho0, double *rho_l, double *rho_v,
                         int32_t *status);

/*
 * lbm_coexistence_many without any device allocation, for callers that
 * cannot allocate device memory (serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors, bit for bit the same
 * densities, for at most LBM_NOALLOC_MAX_RUNS runs (more: INVALID_ARG
 * before any device work).  Its device memory is a fixed library-owned
 * array of about 1.3 MB per GPU (run states, results, case table), held
 * until the process ends; every call on one GPU reuses it, so calls that
 * overlap on the same GPU (from several host threads) race and must be
 * serialised by the caller.  Synchronous; works on the null stream of the
 * current device.
 */
enum { LBM_NOALLOC_MAX_RUNS = 64 };
int lbm_coexistence_many_noalloc(int32_t m, const double *G, const double *tau, const lbm_mrt *mrt,
                                 int32_t psi, double rho0, double *rho_l, double *rho_v,
                                 int32_t *status);

/*
 * Select the collision of a context: mrt = NULL for BGK (the default), else
 * the MRT rates above (copied).  The MRT kernels are compiled for the
 * run-time tiles (tile_x = 0); if the current launch uses a compile-time
 * tile it is reset to the default launch, and lbm_set_launch then refuses
 * compile-time tiles with UNSUPPORTED.  lbm_init_ligament with rho_l or
 * rho_v <= 0 takes the coexistence densities of the selected collision.
 * Captured graphs are rebuilt.  The batched form uses BGK.  UNSUPPORTED for
 * the FP32-rest storage kinds (F16M, BF16M).
 */
int lbm_set_mrt(lbm_ctx *ctx, const lbm_mrt *mrt);

/*
 * Equal-area (mechanical stability) construction for the equation of state
 * of Eq. (7), P = rho c_s^2 + c_s^2 G psi^2 / 2: the densities with
 * P(rho_v) = P(rho_l) = p whose integral of (p - P) psi'/psi^2 between them
 * vanishes.  Host-only arithmetic (no device work); the start of
 * lbm_coexistence.  Errors: INVALID_ARG for G >= -4/rho0 (no coexistence).
 */
int lbm_equal_area(double G, int32_t psi, double rho0, double *rho_l, double *rho_v);

/*
 * Ligament initial condition (Section 3, Fig. 1): a liquid cylinder along
 * `axis` whose radius is modulated by a cosine with an integer number of
 * waves over the period (the paper's sine of 4x/L is not periodic on the
 * domain; its amplitude R0/10 is amp_rel = 0.1):
 *   R(s) = R0 (1 + amp_rel cos(2 pi s / wavelength)), s the axis coordinate,
 *   rho  = (rho_l + rho_v)/2 - (rho_l - rho_v)/2 tanh(2 (r - R(s)) / width),
 *   rho += noise_amp (2U - 1), U = top 53 bits of SplitMix64(seed + node)
 *          / 2^53 (Steele, Lea & Flood 2014; counter-based),
 *   f_a  = w_a rho (equilibrium at rest),
 * r = distance from (c1, c2), the axis position in the cross-section (c1
 * along the lower-numbered in-plane axis).  rho_l <= 0 or rho_v <= 0 means
 * "use lbm_coexistence(G, tau)".  Resets the step counter to 0.
 */
typedef struct {
    int32_t axis;                  /* 0 = x, 1 = y, 2 = z */
    double R0, amp_rel, wavelength; /* R0 > 0, wavelength > 0 */
    double c1, c2;                 /* axis position in node units */
    double width;                  /* tanh width, > 0 */
    double rho_l, rho_v;           /* densities; <= 0 selects coexistence */
    double noise_amp;              /* >= 0 */
    uint64_t seed;
} lbm_ligament;

int lbm_init_ligament(lbm_ctx *ctx, const lbm_ligament *spec);

/*
 * Advance nsteps >= 0 time steps of Eq. (3) with the force of Eq. (5) and
 * the shift of Eq. (6), fused into one kernel per step (psi recomputed for a
 * one-node halo in on-chip memory; pull streaming between two lattices).
 * Asynchronous and stream-ordered; divergence is reported by
 * lbm_diagnostics, not here.
 */
int lbm_step(lbm_ctx *ctx, int64_t nsteps);

/*
 * Export fields of the current state as FP64.  mask: LBM_FIELD_* bits.
 *   rho   [n]      density (Eq. 4)
 *   u     [3][n]   physical velocity (sum_a c_a f_a + F/2) / rho
 *   force [3][n]   Shan-Chen force (Eq. 5)
 *   pop   [19][n]  populations f_a(x, t) in canonical order
 * Pointers of unrequested fields may be NULL.  on_device = 1: the pointers
 * are device pointers (stream-ordered, no sync); 0: host pointers (syncs).
 */
enum { LBM_FIELD_RHO = 1, LBM_FIELD_U = 2, LBM_FIELD_FORCE = 4, LBM_FIELD_POP = 8 };
int lbm_get_fields(lbm_ctx *ctx, uint32_t mask, double *rho, double *u, double *force,
                   double *pop, int32_t on_device);

/* Replace the state by pop[19][n] (canonical FP64, f_a(x, t)); step counter kept. */
int lbm_set_populations(lbm_ctx *ctx, const double *pop, int32_t on_device);

/*
 * Global diagnostics of the current state, reduced in FP64 on the device
 * (wavefront shuffles, per-block partials, fixed-order final pass, so the
 * result is reproducible):
 *   mass = sum rho, mom = sum_x sum_a c_a f_a (equal to the physical total
 *   since the periodic force sums to zero), rho_min, rho_max,
 *   neck_rho = min over the axis coordinate of the max of rho over the
 *   cross-section (axis set by lbm_set_axis, default z),
 *   nonfinite = number of nodes with a non-finite population or rho <= 0.
 * Synchronises.  Returns LBM_ERR_DIVERGED (with *out filled) if nonfinite > 0.
 */
typedef struct {
    int64_t step;
    double mass, mom[3], rho_min, rho_max, neck_rho;
    int64_t nonfinite;
} lbm_diag;

int lbm_diagnostics(lbm_ctx *ctx, lbm_diag *out);

/* Axis along which neck_rho is taken (0 = x, 1 = y, 2 = z). */
int lbm_set_axis(lbm_ctx *ctx, int32_t axis);

/*
 * Asynchronous diagnostics: enqueue the same reduction into a device ring of
 * LBM_DIAG_RING records without synchronising (for break-up detection over
 * long runs).  lbm_read_diag_history copies the records enqueued since the
 * last read (oldest first; at most LBM_DIAG_RING, older ones are
 * overwritten) and synchronises.  *count receives the number copied.
 */
enum { LBM_DIAG_RING = 4096 };
int lbm_record_diag(lbm_ctx *ctx);
int lbm_read_diag_history(lbm_ctx *ctx, lbm_diag *out, int32_t max, int32_t *count);

/*
 * Droplets of the current state (the break-up analysis of Sections 3-4: the
 * ligament pinches into a main drop and satellites): the 6-connected
 * components of {rho > rho_mid} on the periodic grid, labelled on the device
 * with a union-find.  Each component reports its volume (nodes), its mass
 * (sum of rho, FP64; the last bits depend on the order of the device's
 * atomic additions) and its first node, the smallest linear index
 * (z * ny + y) * nx + x it contains.
 *
 * *count receives the number of components; the min(max_out, *count)
 * largest (volume descending, then first node ascending) are copied to out
 * (may be NULL when max_out is 0).  The per-node work arrays live in the
 * spare lattice, which the next lbm_step overwrites anyway: the state is not
 * touched and no device memory is allocated for them; a temporary device
 * table of 24 bytes per component is allocated and freed.  Synchronises.
 */
typedef struct {
    int64_t volume;
    double mass;
    int64_t first_node;
} lbm_droplet;

int lbm_droplets(lbm_ctx *ctx, double rho_mid, lbm_droplet *out, int32_t max_out, int64_t *count);

/* Steps taken since the last lbm_init_ligament. */
int lbm_get_step(const lbm_ctx *ctx, int64_t *step);

/*
 * Set the step counter (>= 0), e.g. when resuming from a checkpoint taken
 * with lbm_get_fields / lbm_get_step: the stochastic rounding of the F16M and
 * BF16M kinds draws its random numbers from (step, node), so a resumed run
 * repeats the uninterrupted one bit for bit only at the same step number.
 * The other kinds do not use it.
 */
int lbm_set_step(lbm_ctx *ctx, int64_t step);

/*
 * Launch shape of the fused step kernel: an x-y tile of tile_x * tile_y
 * nodes (one thread each) marching zchunk planes along z.  Supported tiles:
 * see lbm_list_tiles.  tile_x = 0 selects a tile shaped at run time for the
 * grid, for a workgroup of tile_y threads (512 or 1024): nx split evenly
 * into the fewest tiles at most 128 (512 threads) or 256 (1024) wide, the
 * width rounded up to a multiple of 32 when nx is one (whole rows when nx
 * fits one tile); height balanced over ny with at most tile_y nodes and 64
 * rows.  zchunk >= 1.  The FP64 kernel is slow with 1024 threads (its
 * registers do not fit), the other storages run fastest there on grids of
 * nx >= 128.  A new context starts on the shape cached by lbm_autotune for
 * its grid, else on the default: the run-time tile of 1024 threads (512 for
 * FP64 or nx < 128) and, on grids of 2^22 nodes or more, the z chunk of at
 * least 4 planes that minimises rounds x (chunk + 18), where a round is as
 * many workgroups as the device holds at once (256 for one 1024-thread
 * workgroup per compute unit) and 18 planes charge a round's start-up, the
 * two extra psi planes of each chunk and the tail; smaller grids, which live
 * in the caches, take the chunk that gives about 256 workgroups (down to one
 * plane).  The shape does not change the results (bit for bit); neither does
 * the kernel's choice, per launch, between marching with the tile's loads
 * for plane z + 2 in flight during plane z's collision and the plain march
 * (taken by FP32 and FP64 when a plane has more tiles than the device keeps
 * resident).
 */
typedef struct {
    int32_t tile_x, tile_y, zchunk;
} lbm_launch;

int lbm_set_launch(lbm_ctx *ctx, const lbm_launch *l);
int lbm_get_launch(const lbm_ctx *ctx, lbm_launch *l);
/* Copy up to max supported tiles into out; *count receives the total. */
int lbm_list_tiles(lbm_launch *out, int32_t max, int32_t *count);
/*
 * The default launch for these parameters (as lbm_create would choose it
 * without a cached shape) and, if tile_w / tile_h are not NULL, the run-time
 * tile's width and height on this grid.  The round size comes from the
 * current device; without one it is taken as 256 workgroups.  Errors:
 * INVALID_ARG (params as for lbm_workspace_bytes, out NULL).
 */
int lbm_default_launch(const lbm_params *p, lbm_launch *out, int32_t *tile_w, int32_t *tile_h);

/*
 * HBM layout of one lattice for these parameters: rows are grouped in
 * records of k = *rows_per_record rows, stored [z][y / k][a][y % k][x]
 * (the 19 population segments of k grid rows contiguous; k = 1 is
 * row-interleaved [z][y][a][x]), and *lattice_bytes is the size of one
 * lattice (a context holds two).  k is the smallest power of two whose
 * segment of k nx elements holds 32 KiB when nx is a power of two from 64 to
 * 1024 on grids of 2^22 nodes or more (k <= 32), else 2 KiB (k <= 8); k
 * never exceeds ny (rows beyond ny in the last record are padding).  Either
 * output may be NULL.
 * Errors: INVALID_ARG (params as for lbm_workspace_bytes).
 */
int lbm_lattice_layout(const lbm_params *p, int32_t *rows_per_record, int64_t *lattice_bytes);

/*
 * Autotuner: time the context's launch, the default launch and each
 * supported tile shape with z chunks of 1, 2, 4, ..., 256 planes on this
 * context's grid, pick the fastest, set it, and store it in the JSON cache
 * named by the environment variable LBM_TUNE_CACHE (if set) keyed by device
 * architecture, storage and grid.  Each candidate is timed in the loop
 * lbm_step runs: 2 ceil(steps_per_candidate / 2) steps alternating between
 * the two lattices, after two warm-up steps.  The current lattice is copied
 * to a temporary device buffer first (one lattice, allocated and freed
 * here) and restored at the end, so the state and the step counter are
 * unchanged.  A later lbm_create with the same key takes the cached shape
 * (lbm_get_launch reports it).  Synchronous.
 */
int lbm_autotune(lbm_ctx *ctx, int32_t steps_per_candidate, lbm_launch *best,
                 double *best_mlups);

/*
 * hipGraph capture of the step loop: lbm_step runs whole chunks of
 * `chunk_steps` (even, 0 disables) as one captured graph each.  Needs a
 * non-null stream.  Captured graphs are rebuilt when the launch shape
 * changes and released by lbm_destroy.
 */
int lbm_set_graph_chunk(lbm_ctx *ctx, int32_t chunk_steps);

/* Thread-local message of the last failing call on this thread (static lifetime). */
const char *lbm_last_error(void);

/* Library version string. */
const char *lbm_version(void);

/*
 * Calibration: copy `bytes` (multiple of 16) from src to dst (device
 * pointers) with a plain streaming kernel on `hip_stream`; the HBM ceiling a
 * bandwidth-bound kernel is compared with.
 */
int lbm_device_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

/* ------------------------------------------------------------------------
 * Batched form: many independent ligaments of different grids and
 * parameters advanced by ONE kernel launch per step (a flat list of
 * (case, tile) work items), optionally replayed as a captured hipGraph.
 * All cases share one storage kind.  A case whose diagnostics find a
 * non-finite or non-positive density is frozen: later steps skip it and its
 * state keeps the values of the step at which it was found.
 */
typedef struct lbm_batch lbm_batch;

size_t lbm_batch_workspace_bytes(int32_t ncases, const lbm_params *p);
int lbm_batch_create(int32_t ncases, const lbm_params *p, void *d_workspace, size_t ws_bytes,
                     void *hip_stream, lbm_batch **out);
/*
 * Set up every case (lbm_init_ligament semantics).  The cases whose
 * densities are to come from lbm_coexistence get them from one
 * lbm_coexistence_many run.  A case whose flat interface diverges at its
 * (G, tau) starts frozen with non-finite densities instead of failing the
 * whole batch.
 */
int lbm_batch_init(lbm_batch *b, const lbm_ligament *specs);
/*
 * Advance every case by nsteps (stream-ordered).  Divergence checks run every
 * 1000 steps on the device; the host takes in the flags of a check when the
 * next one is enqueued (waiting for the device to reach it, so the host runs
 * at most one check interval ahead) or at lbm_batch_diagnostics, and from
 * then on launches no workgroups for the cases found frozen (their
 * workgroups would only exit; measured 19% of a step for 13 frozen cases of
 * 64).  Rebuilding the launch list synchronises the stream once.
 */
int lbm_batch_step(lbm_batch *b, int64_t nsteps);
/* Per-case diagnostics (synchronises); frozen cases report nonfinite > 0. */
int lbm_batch_diagnostics(lbm_batch *b, lbm_diag *out);
/* Per-case FP64 export, as lbm_get_fields, for case `index`. */
int lbm_batch_get_fields(lbm_batch *b, int32_t index, uint32_t mask, double *rho, double *u,
                         double *force, double *pop, int32_t on_device);
/* Launch of the batched step (z chunk >= 4; also resets the chunking to
 * uniform chunks).  The default is the run-time tile of 1024 threads (512
 * for FP64), shaped per case, with z chunks of 5 planes. */
int lbm_batch_set_launch(lbm_batch *b, const lbm_launch *l);
/*
 * Autotuner of the batched launch: time each tile shape with uniform z
 * chunks (4, 5, 6, 8, 12, 16, 32, 64 and 128 planes) and with equal-cost
 * chunks of 4, 8, 16 and 32 rounds (lbm_batch_set_chunking) over the whole
 * item list in the loop lbm_batch_step runs (an even number of launches
 * alternating between each case's two lattices, after two warm-up
 * launches), and keep the fastest launch and chunking.  The current
 * lattices of the cases in the launch list are copied to a temporary device
 * buffer first (allocated and freed here) and restored at the end, so the
 * state is unchanged.  *best_mlups counts the nodes of the cases that are
 * not frozen.  Synchronous.
 */
int lbm_batch_autotune(lbm_batch *b, int32_t steps_per_candidate, lbm_launch *best,
                       double *best_mlups);
/*
 * Chunking of the batched launch: rounds = 0 (the default) cuts every case
 * into z chunks of the launch's zchunk; rounds > 0 sizes each case's chunks
 * (at least 4 planes, an even split of its nz) so that every work item costs
 * about the same, tile and ring nodes times planes, and the launch holds
 * about `rounds` times as many items as the device runs at once.  Errors:
 * INVALID_ARG (rounds < 0, or more items than the workspace was sized for).
 */
int lbm_batch_set_chunking(lbm_batch *b, int32_t rounds);
int lbm_batch_set_graph_chunk(lbm_batch *b, int32_t chunk_steps);
int lbm_batch_destroy(lbm_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* LIBLBM_H */
