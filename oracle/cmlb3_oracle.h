/*
 * Plain FP64 CPU oracle of the three-dimensional (D3Q27) extension of the
 * coupled central-moment LB step (arXiv 2504.09024 states the scheme in 2D
 * and only claims that it extends to 3D).  TEST INFRASTRUCTURE ONLY: loaded
 * by the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark, never by the GPU library.  See cmlb3_oracle.c for what is
 * computed and which reading each step takes.
 *
 * Arrays: fields are [nz][ny][nx] (x fastest); populations are
 * [27][nz][ny][nx] with the direction index slowest.  Direction a has
 * components (ex, ey, ez) = (a % 3, (a / 3) % 3, a / 9) mapped through
 * {0, 1, 2} -> {0, +1, -1}.  Central moment k has exponents
 * (k % 3, (k / 3) % 3, k / 9).  All storage is owned by the caller.
 */
#ifndef CMLB3_ORACLE_H
#define CMLB3_ORACLE_H
#include <stdint.h>

#define O3_DIAG_N 30

typedef struct {
    int32_t nx, ny, nz;
    int32_t walls; /* 0: periodic in y, 1: moving walls at y = -1/2, ny - 1/2 */
    int32_t flow;  /* 0 none, 1 prescribed, 2 coupled (as in the 2D oracle) */
    int32_t pad_;
    double W, phi_a, phi_b, M_phi, D_s;
    double rho_a, rho_b, nu_a, nu_b, omega_zeta;
    double sigma0, beta, c_max;
    double u_wall; /* walls move along x at -u_wall (y = -1/2) and +u_wall */
    double F_ext_x, F_ext_y, F_ext_z;
    double vel_period_T;
} o3_params;

void o3_directions(int ex[27], int ey[27], int ez[27]);
void o3_weights(double w[27]);
void o3_central_moments(const double q[27], const double u[3], double out[27]);
void o3_populations_from_central(const double kappa[27], const double u[3], double q[27]);
int o3_populations_from_central_solve(const double kappa[27], const double u[3], double q[27]);
void o3_collide_scalar(const double q[27], const double u[3], double s, const double j[3],
                       double omega1, double qt[27]);
void o3_collide_flow(const double g[27], const double u[3], double P, double rho,
                     const double fp[3], const double ft[3], double omega_zeta, double omega_nu,
                     double gt[27]);
int o3_check_params(const o3_params* p);
int o3_init(const o3_params* p, const double* phi, const double* c, const double* ux,
            const double* uy, const double* uz, const double* P, double* f, double* h,
            double* g);
int o3_step(const o3_params* p, int64_t t, const double* ushape, const double* f,
            const double* h, const double* g, double* f2, double* h2, double* g2);
int o3_run(const o3_params* p, int64_t t0, int64_t nsteps, const double* ushape, double* f,
           double* h, double* g);
int o3_fields(const o3_params* p, int64_t t, const double* ushape, const double* f,
              const double* h, const double* g, double* phi, double* c, double* ux,
              double* uy, double* uz, double* P);

#endif
