/*
 * Plain FP64 CPU oracle of the coupled central-moment LB step
 * (arXiv 2504.09024).  TEST INFRASTRUCTURE ONLY: loaded by the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark, never by the
 * GPU library.  See cmlb_oracle.c for what is computed and which reading of
 * the paper each step takes.
 *
 * Arrays: fields are row-major [ny][nx]; populations are [9][ny][nx] with
 * the direction index slowest.  All storage is owned by the caller.
 */
#ifndef CMLB_ORACLE_H
#define CMLB_ORACLE_H
#include <stdint.h>

#define O_FLOW_NONE 0
#define O_FLOW_PRESCRIBED 1
#define O_FLOW_COUPLED 2
#define O_DIAG_N 22

typedef struct {
    int32_t nx, ny;
    int32_t walls; /* 0: periodic in y, 1: moving walls at y = -1/2, ny - 1/2 */
    int32_t flow;  /* O_FLOW_* */
    int32_t force_abs_grad; /* 0: |grad phi|^2 weight (default), 1: |grad phi| */
    int32_t pad_;
    double W, phi_a, phi_b, M_phi, D_s;
    double rho_a, rho_b, nu_a, nu_b, omega_zeta;
    double sigma0, beta, c_max;
    double u_wall, F_ext_x, F_ext_y;
    double vel_period_T;
} o_params;

int o_num_threads(void);
void o_central_moments(const double q[9], double ux, double uy, double out[9]);
int o_populations_from_central(const double kappa[9], double ux, double uy, double q[9]);
void o_weights(double w[9]);
void o_directions(int ex[9], int ey[9]);
double o_langmuir(double sigma0, double beta, double c_max, double c);
double o_omega_from_transport(double coeff);
int o_collide_scalar(const double q[9], double ux, double uy, double s, double jx, double jy,
                     double omega1, double qt[9]);
int o_collide_flow(const double g[9], double ux, double uy, double P, double rho, double fpx,
                   double fpy, double ftx, double fty, double omega_zeta, double omega_nu,
                   double gt[9]);
int o_check_params(const o_params* p);
int o_init(const o_params* p, const double* phi, const double* c, const double* ux,
           const double* uy, const double* P, double* f, double* h, double* g);
int o_step(const o_params* p, int64_t t, const double* ux_shape, const double* uy_shape,
           const double* f, const double* h, const double* g, double* f2, double* h2,
           double* g2);
int o_run(const o_params* p, int64_t t0, int64_t nsteps, const double* ux_shape,
          const double* uy_shape, double* f, double* h, double* g);
int o_fields(const o_params* p, int64_t t, const double* ux_shape, const double* uy_shape,
             const double* f, const double* h, const double* g, double* phi, double* c,
             double* ux, double* uy, double* P);
int o_node_diag(const o_params* p, int64_t t, const double* ux_shape, const double* uy_shape,
                const double* f, const double* h, const double* g, int x, int y,
                double out[O_DIAG_N]);

#endif
