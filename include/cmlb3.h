/*
 * cmlb3.h -- C ABI of the three-dimensional (D3Q27) form of the coupled
 * central-moment lattice Boltzmann step (Schupbach & Premnath, arXiv
 * 2504.09024).  The paper states the three schemes in 2D (Sec. 3: the
 * interface-bound surfactant lattice h; App. C: the CACE phase-field lattice
 * f; App. D: the two-fluid flow lattice g) and only claims that they extend
 * to 3D.  This library takes each step over to D3Q27 = D1Q3 x D1Q3 x D1Q3
 * by the tensor-product structure of the 2D expressions: equilibria are the
 * 2D ones with a third factor, the flow lattice's second-order trace relaxes
 * at omega_zeta and its deviatoric and off-diagonal parts at omega_nu, the
 * gradients use the D3Q27 weights.
 *
 * Conventions are those of cmlb.h (status codes, precision enum, flow and
 * boundary enums; host I/O in FP64; library-owned device memory;
 * asynchronous cmlb3_step on the context's stream), with:
 *   - fields [nz][ny][nx] (x fastest); populations [27][nz][ny][nx],
 *     direction a = ix + 3 iy + 9 iz with component index 0, 1, 2 meaning
 *     0, +1, -1 (a = 0 is the rest direction);
 *   - x and z periodic; y periodic or moving walls at y = -1/2 (moving at
 *     -u_wall along x) and y = ny - 1/2 (+u_wall).
 */
#ifndef CMLB3_H
#define CMLB3_H

#include <stdint.h>

#include "cmlb.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Parameters of one 3D simulation (lattice units).  Fields as in
 * cmlb_sim_params, plus nz and the z component of the external force. */
typedef struct {
    int32_t nx, ny, nz;
    int32_t bc_y; /* cmlb_bc */
    int32_t flow; /* cmlb_flow */
    int32_t pad_;
    double W, phi_a, phi_b, M_phi, D_s;
    double rho_a, rho_b, nu_a, nu_b, omega_zeta;
    double sigma0, beta, c_max;
    double u_wall, F_ext_x, F_ext_y, F_ext_z;
    double vel_period_T;
} cmlb3_sim_params;

typedef struct cmlb3_ctx cmlb3_ctx;

/* Create a context of n_sims 3D simulations advanced together (two kernel
 * launches per step cover every sim: moments, then collision and store).
 * All sims share flow and bc_y.  Each lattice of each sim must fit 2^31
 * bytes (27 nx ny nz x storage bytes).  Device buffers: two copies of the
 * populations, 18 moment planes per node in the compute type, small
 * tables.  On failure *out is NULL. */
int cmlb3_create(const cmlb3_sim_params* params, int32_t n_sims, int32_t precision,
                 void* hip_stream, cmlb3_ctx** out);

/* Initialise simulation `sim` from host fields ([nz][ny][nx] FP64; phi and c
 * required; u components NULL = 0, the prescribed velocity's spatial shape
 * for CMLB_FLOW_PRESCRIBED; p NULL = rho(phi) cs^2, which with rho_a !=
 * rho_b jumps by cs^2 (rho_a - rho_b) across the interface: a drop meant to
 * start near rest takes a uniform p).  Populations are set to the
 * central-moment equilibria of these fields.  Resets the step counter.
 * Synchronous. */
int cmlb3_init_fields(cmlb3_ctx* ctx, int32_t sim, const double* phi, const double* c,
                      const double* ux, const double* uy, const double* uz, const double* p);

/* Advance every simulation by n_steps >= 0 steps (asynchronous). */
int cmlb3_step(cmlb3_ctx* ctx, int32_t n_steps);

/* Fields at the current step: phi = sum f, c = sum h, u = (sum e g +
 * cs^2 F_t/2)/(cs^2 rho), P = sum g + Gamma/2 (coupled); prescribed u and
 * P = 0 otherwise.  Any pointer may be NULL.  Synchronises; CMLB_ERANGE if a
 * fault flag is set. */
int cmlb3_read_fields(cmlb3_ctx* ctx, int32_t sim, double* phi, double* c, double* ux,
                      double* uy, double* uz, double* p);

/* FP64 totals of phi and c of simulation `sim` (fixed summation order). */
int cmlb3_inventory(cmlb3_ctx* ctx, int32_t sim, double* sum_phi, double* sum_c);

/* Decoded pre-collision populations of `sim` ([27][nz][ny][nx] each; g only
 * when coupled; NULL skips).  Synchronises. */
int cmlb3_get_populations(cmlb3_ctx* ctx, int32_t sim, double* f, double* h, double* g);

/* Overwrite the populations of `sim` (encoded to the storage precision,
 * round to nearest).  f and h required, g when coupled.  Synchronous. */
int cmlb3_set_populations(cmlb3_ctx* ctx, int32_t sim, const double* f, const double* h,
                          const double* g);

/* Fault flags of `sim` (bit 0 non-finite, bit 1 Langmuir domain). */
int cmlb3_fault_flags(cmlb3_ctx* ctx, int32_t sim, int32_t* flags);

/* Block until the context's stream is idle; CMLB_ERANGE if a fault flag is set. */
int cmlb3_synchronize(cmlb3_ctx* ctx);

/* Collision launch shape: columns of 64 x ty nodes (ty waves per
 * workgroup), each marching through zs consecutive z planes.  Accepted
 * (ty, zs) pairs are listed by cmlb3_launch_options; (0, 0) restores the
 * default ((8, 16) with FP32 storage, (4, 8) with FP16 and FP64).  Results
 * do not depend on it (bitwise). */
int cmlb3_set_tile_shape(cmlb3_ctx* ctx, int32_t ty, int32_t zs);
/* Writes up to cap/2 accepted (ty, zs) pairs into shapes[]; returns the count. */
int cmlb3_launch_options(const cmlb3_ctx* ctx, int32_t* shapes, int32_t cap);

/* Cache policy of the collision kernel's population stores, as for
 * cmlb_set_store_policy: 0 (default) non-temporal when the two population
 * buffers together exceed 256 MiB, 1 default stores, 2 non-temporal.
 * Results do not depend on it (bitwise). */
int cmlb3_set_store_policy(cmlb3_ctx* ctx, int32_t policy);

/* Autotuner, as cmlb_autotune: advance the context's own simulations by
 * `steps` (1..100000) steps with every accepted collision shape (see
 * cmlb3_launch_options) under both store policies (1 default, 2
 * non-temporal), timed with HIP events on the context's stream in the
 * context's launch mode (graph replays when graphs are on, after an untimed
 * warm-up that builds the graph), and keep the fastest (written to *ty, *zs,
 * *policy when not NULL).  Every trial starts from a device copy of the
 * populations, restored afterwards together with the step counter and the
 * fault flags: the simulations continue exactly as if no trial had run.
 * Needs one population buffer's worth of free device memory (CMLB_ENOMEM
 * otherwise).  Synchronous.  On error the previous launch configuration and
 * the state are restored. */
int cmlb3_autotune(cmlb3_ctx* ctx, int32_t steps, int32_t* ty, int32_t* zs, int32_t* policy);

/* Replay steps through HIP graphs (1, default) or launch directly (0).
 * Results do not depend on it. */
int cmlb3_set_use_graph(cmlb3_ctx* ctx, int32_t on);

int64_t cmlb3_step_count(const cmlb3_ctx* ctx);
const char* cmlb3_last_error(const cmlb3_ctx* ctx);
void cmlb3_destroy(cmlb3_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* CMLB3_H */
