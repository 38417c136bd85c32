/*
 * cmlb.h -- C ABI of the MI355X-native coupled central-moment lattice
 * Boltzmann step for interface-bound surfactant transport (Schupbach &
 * Premnath, arXiv 2504.09024).
 *
 * One time step advances three coupled D2Q9 population sets per node:
 *   f  -- phase field phi, conservative Allen-Cahn equation
 *         (Eq. CACE; scheme of App. C),
 *   h  -- interface-bound surfactant c with the confining flux
 *         D_s theta_c n (Eq. ISS; scheme of Sec. 3),
 *   g  -- pressure-based two-fluid flow P, u driven by the capillary and
 *         Marangoni force of Eq. Fs with the Langmuir isotherm of Eq. EOS
 *         (scheme of App. D).
 * Each lattice is collided in central moments (raw moments by the matrix P
 * of App. A, central moments by F(u) of App. B, relaxation, back-transform)
 * and streamed.
 *
 * Conventions shared by every call:
 *   - Every function returns CMLB_OK (0) or a negative cmlb_status; no
 *     exception or abort crosses the ABI.  The context keeps a message for
 *     the last error (cmlb_last_error).
 *   - Host arrays are FP64, row-major [ny][nx] (x fastest) for fields and
 *     [9][ny][nx] (direction slowest, D2Q9 order of Eqs. ex/ey with
 *     e_8 = (+1, -1)) for populations.  The library copies them; the caller
 *     keeps ownership.  Whatever the storage precision, host I/O is FP64.
 *   - Device memory is owned by the library (hipMalloc at cmlb_create,
 *     released at cmlb_destroy).
 *   - Work is enqueued on the stream given at cmlb_create (or a stream the
 *     library creates when NULL).  cmlb_step is asynchronous; the calls
 *     that return host data synchronise that stream.
 *   - One context per stream; calls on one context are not thread-safe.
 */
#ifndef CMLB_H
#define CMLB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CMLB_OK = 0,
    CMLB_EINVAL = -1,    /* bad argument, size or parameter */
    CMLB_ENOMEM = -2,    /* device or host allocation failed */
    CMLB_EDEVICE = -3,   /* a HIP call failed (message in cmlb_last_error) */
    CMLB_EUNSTABLE = -4, /* a relaxation rate derived from the parameters is outside (0, 2) */
    CMLB_ERANGE = -5,    /* a fault flag was raised on the device (see cmlb_fault_flags) */
    CMLB_ESTATE = -6     /* call out of order (e.g. step before every sim was initialised) */
} cmlb_status;

/* Storage precision of the populations.  Arithmetic is FP64 for
 * CMLB_FP64 and FP32 otherwise, except that CMLB_FP32 maps the flow
 * lattice's post-collision moments back to populations in FP64 (its stored
 * values then carry only the rounding of the store); inventories are
 * always FP64. */
typedef enum {
    CMLB_FP64 = 0,
    CMLB_FP32 = 1, /* FP32 deviations from the rest state, scaled by 1/w_a */
    CMLB_FP16 = 2  /* IEEE binary16 deviations from the rest state, scaled by 2^k/w_a */
} cmlb_precision;
/* FP16 stores round stochastically; the random word of a store is drawn from
 * the step number and the node's index counted over all simulations of the
 * context, so an FP16 simulation's results depend on its place in the batch
 * (which simulations precede it).  FP64 and FP32 results do not: a
 * simulation advanced inside a batch is bitwise the same as alone. */

typedef enum {
    CMLB_BC_PERIODIC = 0,    /* y periodic */
    CMLB_BC_MOVING_WALLS = 1 /* walls at y = -1/2 (moving at -u_wall) and y = ny - 1/2 (+u_wall) */
} cmlb_bc;

typedef enum {
    CMLB_FLOW_NONE = 0,       /* u = 0; lattices f and h only (Sec. 4.1) */
    CMLB_FLOW_PRESCRIBED = 1, /* u(x, t) = u_shape(x) cos(pi t / T); f and h only (Sec. 4.2) */
    CMLB_FLOW_COUPLED = 2     /* f, h and g coupled through F_s and u (Sec. 4.3) */
} cmlb_flow;

/* Parameters of one simulation, in lattice units (dx = dt = 1).
 * x is always periodic.  Symbols follow the paper:
 *   W           interface width (Eq. CACE, theta)
 *   phi_a/phi_b bulk values of phi, phi_a != phi_b
 *   M_phi       mobility; omega_kappa = 1/(M_phi/cs^2 + 1/2) (App. C)
 *   D_s         surfactant diffusivity; omega_chi = 1/(D_s/cs^2 + 1/2)
 *               (Eq. diffcoeffscalarfield)
 *   rho_a/b, nu_a/b  densities and kinematic viscosities of the two
 *               phases, interpolated linearly in phi (App. D);
 *               omega_nu = 1/(nu/cs^2 + 1/2) per node
 *   omega_zeta  bulk-viscosity relaxation rate (App. D)
 *   sigma0, beta, c_max  Langmuir isotherm sigma = sigma0 (1 + beta ln(1 - c/c_max))
 *   u_wall      wall speed for CMLB_BC_MOVING_WALLS
 *   F_ext_x/y   uniform external body force (coupled flow)
 *   vel_period_T  period factor of the prescribed velocity; 0 = steady
 * Every derived relaxation rate must lie in (0, 2) (else CMLB_EUNSTABLE). */
typedef struct {
    int32_t nx, ny;
    int32_t bc_y; /* cmlb_bc */
    int32_t flow; /* cmlb_flow */
    double W, phi_a, phi_b, M_phi, D_s;
    double rho_a, rho_b, nu_a, nu_b, omega_zeta;
    double sigma0, beta, c_max;
    double u_wall, F_ext_x, F_ext_y;
    double vel_period_T;
} cmlb_sim_params;

typedef struct cmlb_ctx cmlb_ctx;

/* Create a context holding n_sims independent simulations that advance
 * together (one kernel launch per step covers every sim).  All sims must
 * share flow and bc_y; sizes and the other parameters may differ.
 * precision is a cmlb_precision.  hip_stream is a hipStream_t (NULL: the
 * library creates and owns one).  Device buffers: two copies of every
 * population set (f, h, and g when coupled) plus small per-tile tables.
 * One simulation's populations (rows padded to multiples of 64 nodes) must
 * fit 2^31 bytes: 27 or 18 values per node of 8, 4 or 2 bytes (CMLB_EINVAL
 * otherwise; e.g. at most 19.9 M nodes for FP32 coupled flow).  On failure
 * *out is NULL. */
int cmlb_create(const cmlb_sim_params* params, int32_t n_sims, int32_t precision,
                void* hip_stream, cmlb_ctx** out);

/* Initialise simulation `sim` from host fields (each [ny][nx], FP64).
 * phi and c are required.  ux, uy: velocity (NULL = 0); for
 * CMLB_FLOW_PRESCRIBED they are the spatial shape u_shape used every step.
 * p: pressure (NULL = rho(phi) cs^2; with rho_a != rho_b that default
 * jumps by cs^2 (rho_a - rho_b) across the interface, so a drop meant to
 * start near rest takes a uniform p).  Populations are set to the
 * central-moment equilibria of App. C, Sec. 3 and App. D for these fields
 * (the paper initialises the fields only, Sec. 4).  Resets the step
 * counter of the context to 0.  Synchronous. */
int cmlb_init_fields(cmlb_ctx* ctx, int32_t sim, const double* phi, const double* c,
                     const double* ux, const double* uy, const double* p);

/* Advance every simulation by n_steps >= 0 collide-and-stream steps.
 * Asynchronous on the context's stream.  Returns CMLB_ERANGE if a fault
 * flag raised by earlier work was already seen by a synchronising call. */
int cmlb_step(cmlb_ctx* ctx, int32_t n_steps);

/* Fields of simulation `sim` at the current step: phi = sum f, c = sum h,
 * and for coupled flow u = (sum e g + cs^2 F_t/2)/(cs^2 rho) and
 * P = sum g + sigma_00/2 (App. D, last step).  For prescribed flow u is the
 * prescribed velocity at the current step and P = 0; for no flow u = 0 and
 * P = 0.  Any output pointer may be NULL.  Synchronises; returns
 * CMLB_ERANGE if a fault flag is set. */
int cmlb_read_fields(cmlb_ctx* ctx, int32_t sim, double* phi, double* c, double* ux,
                     double* uy, double* p);

/* Totals of phi and of c over simulation `sim` at the current step, summed
 * in FP64 on the device in a fixed order (bitwise reproducible).
 * Synchronises. */
int cmlb_inventory(cmlb_ctx* ctx, int32_t sim, double* sum_phi, double* sum_c);

/* Totals of phi and of c for the n simulations first .. first + n - 1 in
 * one pair of launches (conservative forms of Eqs. CACE and ISS: the
 * zeroth moments of f and h summed over the grid), into sums[2 n] (host,
 * caller-owned): sums[2 i] = total phi and sums[2 i + 1] = total c of
 * simulation first + i.  The order of every FP64 addition is fixed
 * (per row, then rows in order), so each pair is bitwise equal to what
 * cmlb_inventory returns for that simulation alone.  Synchronises.
 * CMLB_EINVAL for an empty or out-of-range simulation range or a NULL
 * sums. */
int cmlb_inventories(cmlb_ctx* ctx, int32_t first, int32_t n, double* sums);

/* Rows of the largest simulation range cmlb_inventories_noalloc accepts. */
#define CMLB_NOALLOC_MAX_ROWS 65536

/* Allocation-free form of cmlb_inventories, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  It enqueues the same two
 * launches on the context's stream and returns without synchronising; it
 * calls no hipMalloc, hipFree or other allocating routine and copies
 * nothing to the host.  The totals go to d_sums, DEVICE memory of 2 n
 * doubles owned by the caller and 8-byte aligned, laid out as in
 * cmlb_inventories and bitwise equal to its results.  The row partials go
 * to a scratch array that the library holds in static device memory, one
 * per GPU (1 MiB, kept until the process ends): the simulations of the
 * range may hold at most CMLB_NOALLOC_MAX_ROWS rows in total (CMLB_EINVAL
 * with a message otherwise).  Every call on one GPU shares that GPU's
 * array, and each call overwrites the partials it uses before reading
 * them; calls whose launches overlap on one GPU (other streams, other
 * contexts or threads) race on it and must be ordered by the caller.
 * CMLB_EINVAL also for a bad range or a NULL or misaligned d_sums;
 * CMLB_EDEVICE if the array's device address could not be obtained. */
int cmlb_inventories_noalloc(cmlb_ctx* ctx, int32_t first, int32_t n, double* d_sums);

/* Copy the populations of simulation `sim` to host (f, h, g each
 * [9][ny][nx] FP64, g ignored unless coupled; NULL skips).  Values are the
 * decoded pre-collision populations of the current step.  Synchronises. */
int cmlb_get_populations(cmlb_ctx* ctx, int32_t sim, double* f, double* h, double* g);

/* Overwrite the populations of simulation `sim` from host FP64 arrays
 * (encoded to the storage precision, round to nearest even).  f and h are
 * required, g when coupled.  Does not change the step counter.
 * Synchronous. */
int cmlb_set_populations(cmlb_ctx* ctx, int32_t sim, const double* f, const double* h,
                         const double* g);

/* Set the step counter (used by the prescribed velocity's time factor). */
int cmlb_set_step_count(cmlb_ctx* ctx, int64_t step);

/* Fault flags of simulation `sim` (bit 0: non-finite value, bit 1: c >= c_max
 * or sigma < 0, Eq. EOS).  Synchronises. */
int cmlb_fault_flags(cmlb_ctx* ctx, int32_t sim, int32_t* flags);

/* Block until all work on the context's stream is done; returns
 * CMLB_ERANGE if any fault flag is set. */
int cmlb_synchronize(cmlb_ctx* ctx);

/* Launch configuration of the step kernel: the workgroup tile is width x
 * rows nodes (width 64: one wavefront across x; 128: two).  Accepted pairs
 * are listed by cmlb_launch_options; (0, 0) restores the default.  Results
 * do not depend on it (bitwise).  cmlb_set_tile_rows(ctx, r) is
 * cmlb_set_tile_shape(ctx, 64, r) (r = 0: the default). */
int cmlb_set_tile_shape(cmlb_ctx* ctx, int32_t width, int32_t rows);
int cmlb_set_tile_rows(cmlb_ctx* ctx, int32_t rows);
/* Writes up to cap/2 accepted (width, rows) pairs into shapes[] as
 * consecutive int32 pairs; returns how many pairs the precision has. */
int cmlb_launch_options(const cmlb_ctx* ctx, int32_t* shapes, int32_t cap);

/* Capture the step loop in a HIP graph (1) or launch kernels directly (0).
 * Default 1.  Results do not depend on it. */
int cmlb_set_use_graph(cmlb_ctx* ctx, int32_t on);

/* Map workgroups to tiles so that each of the GPU's 8 XCDs (separate L2
 * caches) works on a contiguous band of tiles (1, default) or in plain
 * dispatch order (0).  Results do not depend on it. */
int cmlb_set_xcd_remap(cmlb_ctx* ctx, int32_t on);

/* Cache policy of the step kernel's population stores: 0 (default) picks
 * non-temporal stores when the two population buffers together exceed the
 * GPU's last-level cache (256 MiB on MI355X) and default stores otherwise;
 * 1 forces default stores, 2 non-temporal stores.  Results do not depend on
 * it (bitwise). */
int cmlb_set_store_policy(cmlb_ctx* ctx, int32_t policy);

/* Autotuner: advance the context's own simulations by `steps` (1..100000)
 * steps with every accepted tile shape under both store policies (default,
 * non-temporal), time each trial with HIP events on the context's stream in
 * the context's launch mode (graph replays when graphs are on, after an
 * untimed warm-up that builds the graph), and keep the fastest (written to *width, *rows, *policy when not NULL;
 * policy as in cmlb_set_store_policy).  Every trial starts from a device
 * copy of the current state, which is restored afterwards together with the
 * step counter and fault flags: the simulations continue exactly as if no
 * trial had run.  Needs one population buffer's worth of free device memory
 * (CMLB_ENOMEM otherwise).  Synchronous.  On error the previous launch
 * configuration and the state are restored. */
int cmlb_autotune(cmlb_ctx* ctx, int32_t steps, int32_t* width, int32_t* rows, int32_t* policy);

/* Order in which tiles are handed to workgroups: column groups of `group`
 * tiles of 64 columns (all tile rows of one group before the next), or 0
 * for plain row-major order (default).  Results do not depend on it. */
int cmlb_set_tile_order(cmlb_ctx* ctx, int32_t group);

/* Measurement aid, not part of the method: the cost of the two ways of
 * separating time steps on the current device.  *us_grid_sync: microseconds
 * per grid-wide barrier (HIP cooperative groups) among `blocks` workgroups of
 * 256 threads in one cooperative launch looping `iters` times, the barrier a
 * multi-step persistent kernel would need between steps.  *us_graph_node:
 * microseconds per kernel in a HIP graph of 16 dependent launches of an
 * empty kernel of `blocks` workgroups, replayed iters / 16 times, the
 * separation the step graphs use.  blocks 1..1024 (CMLB_EDEVICE when the
 * runtime cannot make the grid resident), iters a multiple of 16 in
 * 16..10^6.  Synchronous, on a private stream; allocates a few bytes. */
int cmlb_launch_costs(int32_t blocks, int32_t iters, double* us_grid_sync, double* us_graph_node);

/* Measurement aid, not part of the method: copy `bytes` of device memory
 * from src to dst on hip_stream (NULL = the default stream), asynchronously,
 * with 16-byte vector loads and stores, four per thread.  nontemporal = 1
 * marks loads and stores non-temporal (streamed past the caches), 0 uses
 * the default cache policy.  The plain-copy bandwidth it reaches is the
 * practical ceiling the step's HBM fraction is read against.  Both pointers
 * must be 16-byte aligned and bytes a multiple of 16 (CMLB_EINVAL
 * otherwise); the caller owns both buffers, which must not overlap. */
int cmlb_copy(const void* src, void* dst, int64_t bytes, int32_t nontemporal, void* hip_stream);

/* Measurement aid, not part of the method: the same copy in structure-of-
 * arrays form.  src and dst each hold `planes` contiguous planes of
 * plane_bytes (plane p at byte offset p * plane_bytes); one thread moves one
 * 16-byte vector of every plane, all loads before the stores, so `planes`
 * read and `planes` write streams are open at once, as in a step over 9 or 27
 * direction planes.  planes must be 9 or 27; alignment, size, policy,
 * ownership and error rules as for cmlb_copy; both buffers must hold
 * planes * plane_bytes.  A plane_bytes that is not a multiple of the
 * 128-byte cache line starts planes inside a line and costs bandwidth. */
int cmlb_copy_planes(const void* src, void* dst, int64_t plane_bytes, int32_t planes,
                     int32_t nontemporal, void* hip_stream);

int64_t cmlb_step_count(const cmlb_ctx* ctx);
int32_t cmlb_num_sims(const cmlb_ctx* ctx);
/* Message of the last error on this context (owned by the context). */
const char* cmlb_last_error(const cmlb_ctx* ctx);
/* Release every device buffer, graph and owned stream.  NULL is a no-op. */
void cmlb_destroy(cmlb_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* CMLB_H */
