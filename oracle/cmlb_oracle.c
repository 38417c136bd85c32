/*
 * Plain FP64 CPU oracle for the coupled central-moment lattice Boltzmann
 * step of Schupbach & Premnath, "A robust lattice Boltzmann method for
 * interface-bound transport of a passive scalar" (arXiv 2504.09024).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or helper with the GPU library.
 *
 * What it computes, in the paper's order (Sec. 3 for the surfactant lattice
 * h, App. C for the phase-field lattice f, App. D for the flow lattice g):
 *
 *   1. zeroth/first moments: phi = sum f, c = sum h, P^ = sum g
 *      (Sec. 3 last step, App. C last step, App. D last step);
 *      rho and nu linear in phi (App. D, last equation).
 *   2. interface geometry from phi: isotropic gradient, unit normal,
 *      sharpening coefficient theta (Eq. CACE and the theta definition),
 *      surfactant confining coefficient theta_c (Eq. ISS), curvature.
 *   3. forces: Langmuir sigma(c) (Eq. EOS), surface-tension force F_s
 *      (Eq. Fs), pressure force F_p = -grad psi (App. D).
 *   4. velocity and pressure from the g moments with the half-force
 *      corrections (App. D, last step).
 *   5. per lattice: central moments BY THEIR DEFINITION (sum over the nine
 *      directions of q (e-u)^m (e-u)^n, Eq. cmscalar), relaxation towards
 *      the equilibria (Sec. 3 for chi, App. C for kappa, App. D for eta with
 *      the bulk/shear split B and the source sigma), and back to
 *      populations by SOLVING the 9x9 linear system "the populations whose
 *      central moments about u are the post-collision ones" with Gaussian
 *      elimination.  The printed matrices P^-1 and F^-1 (App. A, B) are not
 *      used here: tests compare them against this solve.
 *   6. streaming, q(x + e, t+1) = q~(x, t), periodic in x, periodic or
 *      half-way bounce-back moving walls in y.
 *
 * Readings of places where the paper is silent or garbled (each one is
 * listed in the design notes of the repository):
 *   - the x component of e_8 is +1 (the printed list has 0; the printed
 *     P matrix, row 1, and e_y fix it);
 *   - the first-order flow equilibria are -psi u_x, -psi u_y (the only sign
 *     for which the raw first moment is rho cs^2 u, as the velocity update
 *     of App. D requires);
 *   - gradients use the isotropic nine-point stencil
 *     d_i Phi = (1/cs^2) sum_a w_a e_ai Phi(x + e_a); the curvature is the
 *     same stencil applied to the unit normal; n = grad phi/(|grad phi|+eps),
 *     eps = 1e-12;
 *   - ghost values of phi, c and psi^ beyond a wall mirror the fluid rows
 *     about the wall plane; the unit normal at a ghost node is computed from
 *     the ghost values of phi like at any node;
 *   - the surface-tension force of Eq. Fs is multiplied by
 *     k_s = 3W/(8 phi_o^2) so that its integral across a tanh interface is
 *     sigma (an option selects |grad phi| in place of |grad phi|^2 with
 *     k_s = 1/(phi_a - phi_b));
 *   - grad sigma = sigma'(c) grad c with sigma'(c) = -sigma0 beta/(c_max-c);
 *   - F_p uses psi^ = P^ - rho cs^2 built from the bare zeroth moment P^;
 *     the equilibria use P = P^ + sigma_00/2;
 *   - all three collisions use the same velocity u at time n;
 *   - moving walls: half-way bounce-back, wall planes at y = -1/2 and
 *     y = ny - 1/2 moving at -u_wall and +u_wall; g gets the momentum
 *     correction 2 w rho (e . u_w) with rho of the fluid node; f and h
 *     bounce back plainly;
 *   - populations are initialised at the central-moment equilibria of the
 *     given fields.
 *
 * Rest weights w_a are not typed in: they are obtained by solving for the
 * populations whose moments are those of the rest state (1,0,0,cs^2,cs^2,
 * 0,0,0,cs^4).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "cmlb_oracle.h"

/* Planted mistakes.  The test suite checks that its pins catch plausible
 * mistakes by building this file with -DORACLE_PLANT=k, which swaps in one
 * wrong expression; the default build (k = 0) computes the method.  Each
 * PLANT(k) site names its mistake. */
#ifndef ORACLE_PLANT
#define ORACLE_PLANT 0
#endif
#define PLANT(k) (ORACLE_PLANT == (k))

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads an OpenMP region of the oracle uses (1 without OpenMP). */
int o_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* D2Q9 directions, Eqs. ex/ey (x component of direction 8 read as +1). */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* Exponents (m, n) of the nine basis vectors p_0..p_8, Eq. Pi. */
static const int MM[9] = {0, 1, 0, 2, 0, 1, 2, 1, 2};
static const int NN[9] = {0, 0, 1, 0, 2, 1, 1, 2, 2};

static const double CS2 = 1.0 / 3.0;
static const double NORMAL_EPS = 1e-12;

static double ipow(double v, int k) {
    double r = 1.0;
    for (int i = 0; i < k; ++i) r *= v;
    return r;
}

static int opposite(int a) {
    for (int b = 0; b < 9; ++b)
        if (EX[b] == -EX[a] && EY[b] == -EY[a]) return b;
    return -1;
}

/* ---------------------------------------------------------------------- */
/* Moments by definition and their inversion by a linear solve.           */
/* ---------------------------------------------------------------------- */

void o_central_moments(const double q[9], double ux, double uy, double out[9]) {
    for (int k = 0; k < 9; ++k) {
        double s = 0.0;
        for (int a = 0; a < 9; ++a)
            /* plant 11: moments about -u */
            s += q[a] * ipow(EX[a] + (PLANT(11) ? ux : -ux), MM[k]) *
                 ipow(EY[a] + (PLANT(11) ? uy : -uy), NN[k]);
        out[k] = s;
    }
}

/* Gaussian elimination with partial pivoting on a 9x9 system. */
static int solve9(double A[9][9], double b[9], double x[9]) {
    for (int col = 0; col < 9; ++col) {
        int piv = col;
        for (int r = col + 1; r < 9; ++r)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        if (A[piv][col] == 0.0) return -1;
        if (piv != col) {
            for (int c = 0; c < 9; ++c) {
                double t = A[col][c];
                A[col][c] = A[piv][c];
                A[piv][c] = t;
            }
            double t = b[col];
            b[col] = b[piv];
            b[piv] = t;
        }
        for (int r = col + 1; r < 9; ++r) {
            double f = A[r][col] / A[col][col];
            if (f == 0.0) continue;
            for (int c = col; c < 9; ++c) A[r][c] -= f * A[col][c];
            b[r] -= f * b[col];
        }
    }
    for (int r = 8; r >= 0; --r) {
        double s = b[r];
        for (int c = r + 1; c < 9; ++c) s -= A[r][c] * x[c];
        x[r] = s / A[r][r];
    }
    return 0;
}

int o_populations_from_central(const double kappa[9], double ux, double uy, double q[9]) {
    double A[9][9], b[9];
    for (int k = 0; k < 9; ++k) {
        for (int a = 0; a < 9; ++a)
            A[k][a] = ipow(EX[a] - ux, MM[k]) * ipow(EY[a] - uy, NN[k]);
        b[k] = kappa[k];
    }
    return solve9(A, b, q);
}

void o_weights(double w[9]) {
    const double rest[9] = {1.0, 0.0, 0.0, CS2, CS2, 0.0, 0.0, 0.0, CS2 * CS2};
    o_populations_from_central(rest, 0.0, 0.0, w);
}

void o_directions(int ex[9], int ey[9]) {
    for (int a = 0; a < 9; ++a) {
        ex[a] = EX[a];
        ey[a] = EY[a];
    }
}

/* ---------------------------------------------------------------------- */
/* Pointwise closures.                                                    */
/* ---------------------------------------------------------------------- */

double o_langmuir(double sigma0, double beta, double c_max, double c) {
    /* plant 13: decimal instead of natural logarithm */
    return sigma0 * (1.0 + beta * (PLANT(13) ? log10(1.0 - c / c_max) : log(1.0 - c / c_max)));
}

/* plant 5: the transport coefficient taken as tau - 1/2 without 1/cs2 */
double o_omega_from_transport(double coeff) {
    return 1.0 / ((PLANT(5) ? coeff : coeff / CS2) + 0.5);
}

static double lin_phi(const o_params* p, double phi, double va, double vb) {
    return vb + (phi - p->phi_b) / (p->phi_a - p->phi_b) * (va - vb);
}

/* ---------------------------------------------------------------------- */
/* Single-node collisions (Sec. 3, App. C, App. D).                       */
/* ---------------------------------------------------------------------- */

/* Scalar lattices f and h: equilibria (s, J_x, J_y, cs2 s, cs2 s, 0, 0, 0,
 * cs2^2 s) and relaxation diag(1, w1, w1, 1, ..., 1). */
int o_collide_scalar(const double q[9], double ux, double uy, double s, double jx, double jy,
                     double omega1, double qt[9]) {
    double k[9], keq[9], lam[9], kt[9];
    o_central_moments(q, ux, uy, k);
    keq[0] = s;
    keq[1] = jx;
    keq[2] = jy;
    keq[3] = CS2 * s;
    keq[4] = CS2 * s;
    keq[5] = 0.0;
    keq[6] = 0.0;
    keq[7] = 0.0;
    keq[8] = CS2 * CS2 * s;
    for (int i = 0; i < 9; ++i) lam[i] = 1.0;
    lam[1] = omega1;
    lam[2] = omega1;
    for (int i = 0; i < 9; ++i) kt[i] = k[i] + lam[i] * (keq[i] - k[i]);
    return o_populations_from_central(kt, ux, uy, qt);
}

/* Flow lattice g (App. D).  P is the corrected pressure, psi = P - rho cs2,
 * (fpx, fpy) = -grad psi, (ftx, fty) the total force. */
int o_collide_flow(const double g[9], double ux, double uy, double P, double rho, double fpx,
                   double fpy, double ftx, double fty, double omega_zeta, double omega_nu,
                   double gt[9]) {
    double eta[9], eq[9], src[9];
    o_central_moments(g, ux, uy, eta);
    const double psi = P - rho * CS2;
    const double ux2 = ux * ux, uy2 = uy * uy;
    eq[0] = P;
    /* plant 2: the first-order equilibria with the sign as printed */
    eq[1] = (PLANT(2) ? psi : -psi) * ux;
    eq[2] = (PLANT(2) ? psi : -psi) * uy;
    eq[3] = CS2 * P + psi * ux2;
    eq[4] = CS2 * P + psi * uy2;
    eq[5] = psi * ux * uy;
    eq[6] = -psi * (ux2 + CS2) * uy;
    eq[7] = -psi * (uy2 + CS2) * ux;
    eq[8] = CS2 * CS2 * CS2 * rho + psi * (ux2 + CS2) * (uy2 + CS2);
    const double gam = fpx * ux + fpy * uy;
    src[0] = gam;
    src[1] = CS2 * ftx - ux * gam;
    src[2] = CS2 * fty - uy * gam;
    /* plant 3: factor 2 of the diagonal second-order sources dropped */
    src[3] = (PLANT(3) ? 1.0 : 2.0) * CS2 * fpx * ux + (ux2 + CS2) * gam;
    src[4] = (PLANT(3) ? 1.0 : 2.0) * CS2 * fpy * uy + (uy2 + CS2) * gam;
    src[5] = CS2 * (fpx * uy + fpy * ux) + ux * uy * gam;
    src[6] = 0.0;
    src[7] = 0.0;
    src[8] = 0.0;

    /* B: replace the two diagonal second-order moments by their sum and
     * difference (Eq. combinedforms); identity on the others. */
    double B[9][9];
    memset(B, 0, sizeof(B));
    for (int i = 0; i < 9; ++i) B[i][i] = 1.0;
    B[3][3] = 1.0;
    B[3][4] = 1.0;
    B[4][3] = 1.0;
    B[4][4] = -1.0;
    double eh[9], eqh[9], sh[9];
    for (int i = 0; i < 9; ++i) {
        eh[i] = eqh[i] = sh[i] = 0.0;
        for (int j = 0; j < 9; ++j) {
            eh[i] += B[i][j] * eta[j];
            eqh[i] += B[i][j] * eq[j];
            sh[i] += B[i][j] * src[j];
        }
    }
    double lam[9];
    for (int i = 0; i < 9; ++i) lam[i] = 1.0;
    /* plant 17: the sum of the diagonal moments relaxed at the shear rate */
    lam[3] = PLANT(17) ? omega_nu : omega_zeta;
    lam[4] = omega_nu;
    lam[5] = omega_nu;
    double th[9];
    for (int i = 0; i < 9; ++i) th[i] = eh[i] + lam[i] * (eqh[i] - eh[i]) + (1.0 - 0.5 * lam[i]) * sh[i];
    /* B^-1: bare second-order moments from their sum and difference. */
    double tb[9];
    for (int i = 0; i < 9; ++i) tb[i] = th[i];
    /* plant 4: B^-1 without its factor 1/2 */
    tb[3] = (PLANT(4) ? 1.0 : 0.5) * (th[3] + th[4]);
    tb[4] = (PLANT(4) ? 1.0 : 0.5) * (th[3] - th[4]);
    return o_populations_from_central(tb, ux, uy, gt);
}

/* ---------------------------------------------------------------------- */
/* Whole-grid helpers.                                                    */
/* ---------------------------------------------------------------------- */

#define IDX(p, x, y) ((size_t)(y) * (size_t)(p)->nx + (size_t)(x))
#define POP(arr, p, a, x, y) ((arr)[(size_t)(a) * (size_t)(p)->nx * (size_t)(p)->ny + IDX(p, x, y)])

/* Map a possibly out-of-range coordinate to the grid node whose value the
 * ghost carries: periodic wrap in x; in y periodic wrap or mirror about the
 * wall plane (ghost row -1-k carries row k). */
static int wrap_x(const o_params* p, int x) {
    int n = p->nx;
    x %= n;
    if (x < 0) x += n;
    return x;
}
static int wrap_y(const o_params* p, int y) {
    int n = p->ny;
    if (p->walls) {
        while (y < 0 || y >= n) {
            if (y < 0) y = -1 - y;
            if (y >= n) y = 2 * n - 1 - y;
        }
        return y;
    }
    y %= n;
    if (y < 0) y += n;
    return y;
}

/* Isotropic gradient of a field at node (x, y), ghosts as above. */
static void grad_field(const o_params* p, const double* F, const double w[9], int x, int y,
                       double* gx, double* gy) {
    double sx = 0.0, sy = 0.0;
    for (int a = 0; a < 9; ++a) {
        double v = F[IDX(p, wrap_x(p, x + EX[a]), wrap_y(p, y + EY[a]))];
        sx += w[a] * EX[a] * v;
        sy += w[a] * EY[a] * v;
    }
    /* plant 6: the factor 1/cs2 of the isotropic gradient dropped */
    *gx = PLANT(6) ? sx : sx / CS2;
    *gy = PLANT(6) ? sy : sy / CS2;
}

/* Per-node macroscopic and geometric state at time n. */
typedef struct {
    double phi, c, P_hat, jx, jy;
    double rho, nu;
    double gphix, gphiy, gmag, nx, ny;
    double theta, theta_c, curv;
    double gcx, gcy, gpsix, gpsiy;
    double sigma, fsx, fsy, ftx, fty;
    double ux, uy, P;
    int fault;
} node_state;

/* Work arrays: phi, c, P^, psi^ and the unit normal over the grid. */
typedef struct {
    double *phi, *c, *phat, *psih, *nrmx, *nrmy;
} fields_t;

/* The unit-normal arrays carry one extra row below and above the grid
 * (rows -1 and ny): at a wall the curvature stencil needs the normal at the
 * ghost row, which is computed from the ghost values of phi like at any
 * other node (so its wall-normal component is mirrored too). */
#define NRM(F, p, x, y) ((F)->nrmx[(size_t)((y) + 1) * (size_t)(p)->nx + (size_t)(x)])
#define NRMY(F, p, x, y) ((F)->nrmy[(size_t)((y) + 1) * (size_t)(p)->nx + (size_t)(x)])

static void fields_alloc(const o_params* p, fields_t* F) {
    size_t n = (size_t)p->nx * p->ny;
    size_t ne = (size_t)p->nx * (p->ny + 2);
    F->phi = calloc(n, sizeof(double));
    F->c = calloc(n, sizeof(double));
    F->phat = calloc(n, sizeof(double));
    F->psih = calloc(n, sizeof(double));
    F->nrmx = calloc(ne, sizeof(double));
    F->nrmy = calloc(ne, sizeof(double));
}
static void fields_free(fields_t* F) {
    free(F->phi);
    free(F->c);
    free(F->phat);
    free(F->psih);
    free(F->nrmx);
    free(F->nrmy);
}

static double time_factor(const o_params* p, int64_t t) {
    if (p->vel_period_T == 0.0) return 1.0;
    return cos(M_PI * (double)t / p->vel_period_T);
}

/* Steps 1-2 over the whole grid: zeroth moments and the unit normal. */
static void compute_fields(const o_params* p, const double w[9], const double* f,
                           const double* h, const double* g, fields_t* F) {
    const int nx = p->nx, ny = p->ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double sf = 0.0, sh = 0.0, sg = 0.0;
            for (int a = 0; a < 9; ++a) {
                sf += POP(f, p, a, x, y);
                sh += POP(h, p, a, x, y);
                if (g) sg += POP(g, p, a, x, y);
            }
            F->phi[IDX(p, x, y)] = sf;
            F->c[IDX(p, x, y)] = sh;
            F->phat[IDX(p, x, y)] = sg;
            double rho = lin_phi(p, sf, p->rho_a, p->rho_b);
            /* plant 16: F_p from P^ instead of psi^ = P^ - rho cs2 */
            F->psih[IDX(p, x, y)] = PLANT(16) ? sg : sg - rho * CS2;
        }
#pragma omp parallel for schedule(static)
    for (int y = -1; y <= ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double gx, gy;
            grad_field(p, F->phi, w, x, y, &gx, &gy);
            double mag = sqrt(gx * gx + gy * gy);
            NRM(F, p, x, y) = gx / (mag + NORMAL_EPS);
            NRMY(F, p, x, y) = gy / (mag + NORMAL_EPS);
        }
}

/* Divergence of the unit normal with the isotropic stencil.  Rows -1 and ny
 * are the ghost rows; in y-periodic grids they equal rows ny-1 and 0. */
static double curvature(const o_params* p, const fields_t* F, const double w[9], int x, int y) {
    double s = 0.0;
    for (int a = 0; a < 9; ++a) {
        int xs = wrap_x(p, x + EX[a]);
        int ys = y + EY[a];
        s += w[a] * (EX[a] * NRM(F, p, xs, ys) + EY[a] * NRMY(F, p, xs, ys));
    }
    /* plant 7: curvature with the opposite sign */
    return (PLANT(7) ? -s : s) / CS2;
}

/* Steps 2-4 at one node. */
static void node_macros(const o_params* p, const double w[9], const fields_t* F,
                        const double* g, const double* ux_shape, const double* uy_shape,
                        int64_t t, int x, int y, node_state* s) {
    memset(s, 0, sizeof(*s));
    const size_t i = IDX(p, x, y);
    s->phi = F->phi[i];
    s->c = F->c[i];
    s->P_hat = F->phat[i];
    s->rho = lin_phi(p, s->phi, p->rho_a, p->rho_b);
    /* plant 18: the two viscosities interchanged */
    s->nu = PLANT(18) ? lin_phi(p, s->phi, p->nu_b, p->nu_a) : lin_phi(p, s->phi, p->nu_a, p->nu_b);

    grad_field(p, F->phi, w, x, y, &s->gphix, &s->gphiy);
    s->gmag = sqrt(s->gphix * s->gphix + s->gphiy * s->gphiy);
    s->nx = NRM(F, p, x, y);
    s->ny = NRMY(F, p, x, y);
    const double dphi = p->phi_a - p->phi_b;
    const double phim = 0.5 * (p->phi_a + p->phi_b);
    /* plant 10: sharpening flux dropped; plant 9: confining coefficient 4/W */
    s->theta = PLANT(10) ? 0.0 : (4.0 / p->W) * (p->phi_a - s->phi) * (s->phi - p->phi_b) / dphi;
    s->theta_c = ((PLANT(9) ? 4.0 : 8.0) * s->c / p->W) * (phim - s->phi) / dphi;

    if (p->flow == O_FLOW_COUPLED) {
        /* curvature: divergence of the unit normal, same stencil */
        s->curv = curvature(p, F, w, x, y);
        grad_field(p, F->c, w, x, y, &s->gcx, &s->gcy);
        grad_field(p, F->psih, w, x, y, &s->gpsix, &s->gpsiy);

        double arg = 1.0 - s->c / p->c_max;
        s->sigma = o_langmuir(p->sigma0, p->beta, p->c_max, s->c);
        if (!(arg > 0.0) || !(s->sigma >= 0.0)) s->fault |= 2;
        double dsig = -p->sigma0 * p->beta / (p->c_max - s->c);
        double gsx = dsig * s->gcx, gsy = dsig * s->gcy;
        double nd = s->nx * gsx + s->ny * gsy;
        /* plant 15: normal part added instead of removed */
        double tsx = PLANT(15) ? gsx + s->nx * nd : gsx - s->nx * nd;
        double tsy = PLANT(15) ? gsy + s->ny * nd : gsy - s->ny * nd;
        double weight, ks;
        const double phio = 0.5 * dphi;
        if (p->force_abs_grad) {
            /* plant 19: |grad phi|^2 kept in the |grad phi| reading;
             * plant 20: its normalisation 1/(phi_a - phi_b) dropped */
            weight = PLANT(19) ? s->gmag * s->gmag : s->gmag;
            ks = PLANT(20) ? 1.0 : 1.0 / dphi;
        } else {
            weight = s->gmag * s->gmag;
            /* plant 1: F_s without the normalisation k_s */
            ks = PLANT(1) ? 1.0 : 3.0 * p->W / (8.0 * phio * phio);
        }
        s->fsx = ks * weight * (-s->sigma * s->curv * s->nx + tsx);
        s->fsy = ks * weight * (-s->sigma * s->curv * s->ny + tsy);
        s->ftx = s->fsx + p->F_ext_x;
        s->fty = s->fsy + p->F_ext_y;

        double jx = 0.0, jy = 0.0;
        for (int a = 0; a < 9; ++a) {
            jx += EX[a] * POP(g, p, a, x, y);
            jy += EY[a] * POP(g, p, a, x, y);
        }
        s->jx = jx;
        s->jy = jy;
        /* plant 14: velocity without the half-force correction */
        s->ux = (jx + (PLANT(14) ? 0.0 : 0.5) * CS2 * s->ftx) / (CS2 * s->rho);
        s->uy = (jy + (PLANT(14) ? 0.0 : 0.5) * CS2 * s->fty) / (CS2 * s->rho);
        double fpx = -s->gpsix, fpy = -s->gpsiy;
        s->P = s->P_hat + 0.5 * (fpx * s->ux + fpy * s->uy);
    } else if (p->flow == O_FLOW_PRESCRIBED) {
        double tf = time_factor(p, t);
        s->ux = ux_shape[i] * tf;
        s->uy = uy_shape[i] * tf;
        s->P = 0.0;
    } else {
        s->ux = 0.0;
        s->uy = 0.0;
        s->P = 0.0;
    }
    if (!isfinite(s->phi) || !isfinite(s->c) || !isfinite(s->ux) || !isfinite(s->uy) ||
        !isfinite(s->P))
        s->fault |= 1;
}

int o_check_params(const o_params* p) {
    if (p->nx < 4 || p->ny < 4) return -1;
    if (!(p->phi_a != p->phi_b)) return -1;
    if (!(p->W > 0.0)) return -1;
    double wk = o_omega_from_transport(p->M_phi), wc = o_omega_from_transport(p->D_s);
    if (!(wk > 0.0 && wk < 2.0) || !(wc > 0.0 && wc < 2.0)) return -2;
    if (p->flow == O_FLOW_COUPLED) {
        double w1 = o_omega_from_transport(p->nu_a), w2 = o_omega_from_transport(p->nu_b);
        if (!(w1 > 0.0 && w1 < 2.0) || !(w2 > 0.0 && w2 < 2.0)) return -2;
        if (!(p->omega_zeta > 0.0 && p->omega_zeta < 2.0)) return -2;
        if (!(p->rho_a > 0.0 && p->rho_b > 0.0)) return -1;
        if (!(p->c_max > 0.0)) return -1;
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Initialisation: populations at the central-moment equilibria.          */
/* ---------------------------------------------------------------------- */

int o_init(const o_params* p, const double* phi, const double* c, const double* ux,
           const double* uy, const double* P, double* f, double* h, double* g) {
    if (o_check_params(p) != 0) return -1;
    double w[9];
    o_weights(w);
    const int nx = p->nx, ny = p->ny;
    fields_t F;
    fields_alloc(p, &F);
    memcpy(F.phi, phi, sizeof(double) * nx * ny);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double gx, gy;
            grad_field(p, F.phi, w, x, y, &gx, &gy);
            double mag = sqrt(gx * gx + gy * gy);
            NRM(&F, p, x, y) = gx / (mag + NORMAL_EPS);
            NRMY(&F, p, x, y) = gy / (mag + NORMAL_EPS);
        }
    const double dphi = p->phi_a - p->phi_b, phim = 0.5 * (p->phi_a + p->phi_b);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t i = IDX(p, x, y);
            double u = ux ? ux[i] : 0.0, v = uy ? uy[i] : 0.0;
            double ph = phi[i], cc = c[i];
            double nxv = NRM(&F, p, x, y), nyv = NRMY(&F, p, x, y);
            double theta = (4.0 / p->W) * (p->phi_a - ph) * (ph - p->phi_b) / dphi;
            double theta_c = (8.0 * cc / p->W) * (phim - ph) / dphi;
            double kf[9], kh[9], qf[9], qh[9];
            double keq_f[9] = {ph, p->M_phi * theta * nxv, p->M_phi * theta * nyv, CS2 * ph,
                               CS2 * ph, 0.0, 0.0, 0.0, CS2 * CS2 * ph};
            double keq_h[9] = {cc, p->D_s * theta_c * nxv, p->D_s * theta_c * nyv, CS2 * cc,
                               CS2 * cc, 0.0, 0.0, 0.0, CS2 * CS2 * cc};
            memcpy(kf, keq_f, sizeof(kf));
            memcpy(kh, keq_h, sizeof(kh));
            bad |= o_populations_from_central(kf, u, v, qf) != 0;
            bad |= o_populations_from_central(kh, u, v, qh) != 0;
            for (int a = 0; a < 9; ++a) {
                POP(f, p, a, x, y) = qf[a];
                POP(h, p, a, x, y) = qh[a];
            }
            if (p->flow == O_FLOW_COUPLED && g) {
                double rho = lin_phi(p, ph, p->rho_a, p->rho_b);
                double Pv = P ? P[i] : rho * CS2;
                double psi = Pv - rho * CS2;
                double u2 = u * u, v2 = v * v;
                double eq[9] = {Pv,
                                -psi * u,
                                -psi * v,
                                CS2 * Pv + psi * u2,
                                CS2 * Pv + psi * v2,
                                psi * u * v,
                                -psi * (u2 + CS2) * v,
                                -psi * (v2 + CS2) * u,
                                CS2 * CS2 * CS2 * rho + psi * (u2 + CS2) * (v2 + CS2)};
                double qg[9];
                bad |= o_populations_from_central(eq, u, v, qg) != 0;
                for (int a = 0; a < 9; ++a) POP(g, p, a, x, y) = qg[a];
            }
        }
    fields_free(&F);
    return bad ? -3 : 0;
}

/* ---------------------------------------------------------------------- */
/* One time step.                                                         */
/* ---------------------------------------------------------------------- */

int o_step(const o_params* p, int64_t t, const double* ux_shape, const double* uy_shape,
           const double* f, const double* h, const double* g, double* f2, double* h2,
           double* g2) {
    if (o_check_params(p) != 0) return -1;
    double w[9];
    o_weights(w);
    const int nx = p->nx, ny = p->ny;
    const int coupled = p->flow == O_FLOW_COUPLED;
    fields_t F;
    fields_alloc(p, &F);
    compute_fields(p, w, f, h, coupled ? g : NULL, &F);
    const double omega_k = o_omega_from_transport(p->M_phi);
    const double omega_c = o_omega_from_transport(p->D_s);
    int fault = 0;
#pragma omp parallel for schedule(static) reduction(| : fault)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            node_state s;
            node_macros(p, w, &F, g, ux_shape, uy_shape, t, x, y, &s);
            fault |= s.fault;
            double qf[9], qh[9], qg[9], tf[9], th[9], tg[9];
            for (int a = 0; a < 9; ++a) {
                qf[a] = POP(f, p, a, x, y);
                qh[a] = POP(h, p, a, x, y);
            }
            int bad = 0;
            bad |= o_collide_scalar(qf, s.ux, s.uy, s.phi, p->M_phi * s.theta * s.nx,
                                    p->M_phi * s.theta * s.ny, omega_k, tf);
            bad |= o_collide_scalar(qh, s.ux, s.uy, s.c, p->D_s * s.theta_c * s.nx,
                                    p->D_s * s.theta_c * s.ny, omega_c, th);
            if (coupled) {
                for (int a = 0; a < 9; ++a) qg[a] = POP(g, p, a, x, y);
                double omega_nu = o_omega_from_transport(s.nu);
                bad |= o_collide_flow(qg, s.ux, s.uy, s.P, s.rho, -s.gpsix, -s.gpsiy, s.ftx,
                                      s.fty, p->omega_zeta, omega_nu, tg);
            }
            if (bad) fault |= 4;
            /* streaming: q(x + e, t + 1) = q~(x, t) */
            for (int a = 0; a < 9; ++a) {
                /* plant 12: streamed against the direction */
                int xd = wrap_x(p, x + (PLANT(12) ? -EX[a] : EX[a]));
                int yd = y + (PLANT(12) ? -EY[a] : EY[a]);
                int ad = a;
                double corr = 0.0;
                if (p->walls && (yd < 0 || yd >= ny)) {
                    /* half-way bounce-back into the opposite direction */
                    ad = opposite(a);
                    xd = x;
                    double uw = (yd < 0) ? -p->u_wall : p->u_wall;
                    /* plant 8: correction with the incoming direction */
                    corr = 2.0 * w[ad] * s.rho * (EX[PLANT(8) ? a : ad] * uw);
                    yd = y;
                } else {
                    yd = wrap_y(p, yd);
                }
                POP(f2, p, ad, xd, yd) = tf[a];
                POP(h2, p, ad, xd, yd) = th[a];
                if (coupled) POP(g2, p, ad, xd, yd) = tg[a] + corr;
            }
        }
    fields_free(&F);
    return fault;
}

int o_run(const o_params* p, int64_t t0, int64_t nsteps, const double* ux_shape,
          const double* uy_shape, double* f, double* h, double* g) {
    const size_t n = (size_t)9 * p->nx * p->ny;
    double* f2 = malloc(n * sizeof(double));
    double* h2 = malloc(n * sizeof(double));
    double* g2 = g ? malloc(n * sizeof(double)) : NULL;
    int fault = 0;
    for (int64_t s = 0; s < nsteps; ++s) {
        fault |= o_step(p, t0 + s, ux_shape, uy_shape, f, h, g, f2, h2, g2);
        memcpy(f, f2, n * sizeof(double));
        memcpy(h, h2, n * sizeof(double));
        if (g) memcpy(g, g2, n * sizeof(double));
        if (fault) break;
    }
    free(f2);
    free(h2);
    free(g2);
    return fault;
}

/* Fields at step t: phi, c, u and P as defined by the macroscopic updates. */
int o_fields(const o_params* p, int64_t t, const double* ux_shape, const double* uy_shape,
             const double* f, const double* h, const double* g, double* phi, double* c,
             double* ux, double* uy, double* P) {
    double w[9];
    o_weights(w);
    const int coupled = p->flow == O_FLOW_COUPLED;
    fields_t F;
    fields_alloc(p, &F);
    compute_fields(p, w, f, h, coupled ? g : NULL, &F);
    int fault = 0;
#pragma omp parallel for schedule(static) reduction(| : fault)
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            node_state s;
            node_macros(p, w, &F, g, ux_shape, uy_shape, t, x, y, &s);
            fault |= s.fault;
            size_t i = IDX(p, x, y);
            if (phi) phi[i] = s.phi;
            if (c) c[i] = s.c;
            if (ux) ux[i] = s.ux;
            if (uy) uy[i] = s.uy;
            if (P) P[i] = coupled ? s.P : 0.0;
        }
    fields_free(&F);
    return fault;
}

/* Diagnostics at one node (forces, curvature, ...) for the pin tests. */
int o_node_diag(const o_params* p, int64_t t, const double* ux_shape, const double* uy_shape,
                const double* f, const double* h, const double* g, int x, int y,
                double out[O_DIAG_N]) {
    double w[9];
    o_weights(w);
    fields_t F;
    fields_alloc(p, &F);
    compute_fields(p, w, f, h, p->flow == O_FLOW_COUPLED ? g : NULL, &F);
    node_state s;
    node_macros(p, w, &F, g, ux_shape, uy_shape, t, x, y, &s);
    fields_free(&F);
    double v[O_DIAG_N] = {s.phi,   s.c,   s.P_hat, s.rho,   s.nu,  s.gphix, s.gphiy,
                          s.nx,    s.ny,  s.theta, s.theta_c, s.curv, s.gcx, s.gcy,
                          s.gpsix, s.gpsiy, s.sigma, s.fsx,  s.fsy, s.ux,    s.uy,
                          s.P};
    memcpy(out, v, sizeof(v));
    return s.fault;
}
