/*
 * Plain FP64 CPU oracle of the three-dimensional (D3Q27) form of the coupled
 * central-moment lattice Boltzmann step of arXiv 2504.09024.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously-correct reference
 * the GPU library's 3D path is checked against; only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it.  It shares
 * no code, header, table or helper with the GPU library (nor with the 2D
 * oracle, which the tests use to pin it).
 *
 * The paper states its schemes in 2D (D2Q9: Sec. 3 for the surfactant
 * lattice h, App. C for the phase-field lattice f, App. D for the flow
 * lattice g) and only claims the extension to 3D.  This file takes each 2D
 * step to D3Q27 = D1Q3 x D1Q3 x D1Q3 in the way the 2D expressions factor
 * (every reading is listed in the design notes of the repository):
 *   - directions are the 27 products of {0, +1, -1}; the weights are the
 *     populations of the rest state, obtained by a 27x27 solve;
 *   - central moments are the definition sums
 *     k_abc = sum_q q (ex-ux)^a (ey-uy)^b (ez-uz)^c, a, b, c in {0, 1, 2};
 *   - scalar lattices (f: CACE, h: surfactant): the equilibria are
 *     s prod_i c(a_i) with c = (1, 0, cs2) except the first-order ones,
 *     which are the flux J = M theta n (f) or D_s theta_c n (h); the
 *     first-order moments relax at omega, all others at 1 (the 2D
 *     equilibria are exactly this product with two factors);
 *   - flow lattice: eta_eq = psi prod_i m(a_i, u_i) + rho cs2 prod_i c(a_i)
 *     with m = (1, -u, cs2 + u^2), psi = P - rho cs2 (the 2D equilibria of
 *     App. D, with the first-order sign read as -psi u, are this product);
 *     the source has the 2D structure: sigma_0 = Gamma = F_p.u,
 *     sigma_i = cs2 F_t,i - u_i Gamma, sigma_ii = 2 cs2 F_p,i u_i +
 *     (u_i^2 + cs2) Gamma, sigma_ij = cs2 (F_p,i u_j + F_p,j u_i) +
 *     u_i u_j Gamma, zero from third order on; the trace of the second-order
 *     moments relaxes at omega_zeta, their deviatoric part and the
 *     off-diagonal ones at omega_nu, everything else at 1;
 *   - back to populations: the moment map is a tensor product of one-axis
 *     maps, so it is inverted axis by axis (central -> raw:
 *     r0 = k0, r1 = k1 + u k0, r2 = k2 + 2u k1 + u^2 k0; raw -> populations:
 *     q0 = r0 - r2, q+ = (r2 + r1)/2, q- = (r2 - r1)/2); the tests check
 *     this against a dense 27x27 solve;
 *   - gradients: d_i Phi = (1/cs2) sum_a w_a e_ai Phi(x + e_a) with the
 *     D3Q27 weights; n = grad phi/(|grad phi| + 1e-12); curvature = the same
 *     stencil applied to n; F_s = k_s |grad phi|^2 (-sigma K n + grad_s
 *     sigma), k_s = 3W/(8 phi_o^2);
 *   - x and z periodic; y periodic or half-way bounce-back walls at
 *     y = -1/2 (moving at -u_wall along x) and y = ny - 1/2 (+u_wall), g
 *     corrected by 2 w rho (e . u_w); ghost phi, c, psi^ mirror the fluid
 *     planes about the wall and the ghost normal is computed from the ghost
 *     phi, as in the 2D oracle;
 *   - velocity u = (sum e g + cs2 F_t/2)/(cs2 rho), P = P^ + Gamma/2, all
 *     at time n; populations initialised at the equilibria of the fields.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "cmlb3_oracle.h"

/* Planted mistakes (see cmlb_oracle.c): built with -DORACLE_PLANT=k for the
 * test suite's check of its pins; the default build computes the method. */
#ifndef ORACLE_PLANT
#define ORACLE_PLANT 0
#endif
#define PLANT(k) (ORACLE_PLANT == (k))

#ifdef _OPENMP
#include <omp.h>
#endif

static const double CS2 = 1.0 / 3.0;
static const double NORMAL_EPS = 1e-12;
static const int E1[3] = {0, 1, -1};

static int ex_of(int a) { return E1[a % 3]; }
static int ey_of(int a) { return E1[(a / 3) % 3]; }
static int ez_of(int a) { return E1[a / 9]; }

static double ipow(double v, int k) {
    double r = 1.0;
    for (int i = 0; i < k; ++i) r *= v;
    return r;
}

static int opposite(int a) {
    for (int b = 0; b < 27; ++b)
        if (ex_of(b) == -ex_of(a) && ey_of(b) == -ey_of(a) && ez_of(b) == -ez_of(a)) return b;
    return -1;
}

void o3_directions(int ex[27], int ey[27], int ez[27]) {
    for (int a = 0; a < 27; ++a) {
        ex[a] = ex_of(a);
        ey[a] = ey_of(a);
        ez[a] = ez_of(a);
    }
}

/* ---------------------------------------------------------------------- */
/* Moments by definition and their inversion.                             */
/* ---------------------------------------------------------------------- */

void o3_central_moments(const double q[27], const double u[3], double out[27]) {
    for (int k = 0; k < 27; ++k) {
        const int mx = k % 3, my = (k / 3) % 3, mz = k / 9;
        double s = 0.0;
        for (int a = 0; a < 27; ++a)
            s += q[a] * ipow(ex_of(a) - u[0], mx) * ipow(ey_of(a) - u[1], my) *
                 ipow(ez_of(a) - u[2], mz);
        out[k] = s;
    }
}

/* One axis of the inverse: three central moments (exponents 0, 1, 2 along
 * the axis) to the three populations (e = 0, +1, -1 along the axis). */
static void axis_inverse(double k0, double k1, double k2, double u, double out[3]) {
    const double r0 = k0, r1 = k1 + u * k0, r2 = k2 + 2.0 * u * k1 + u * u * k0;
    out[0] = r0 - r2;
    /* plant 22: the two moving populations swapped */
    out[PLANT(22) ? 2 : 1] = 0.5 * (r2 + r1);
    out[PLANT(22) ? 1 : 2] = 0.5 * (r2 - r1);
}

void o3_populations_from_central(const double kappa[27], const double u[3], double q[27]) {
    /* t[i + 3j + 9k]: index i is the x population (after the x pass) or the x
     * moment exponent (before), likewise j for y and k for z. */
    double t[27], s[27], o[3];
    memcpy(t, kappa, sizeof(t));
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) {
            const int b = 3 * j + 9 * k;
            axis_inverse(t[b], t[b + 1], t[b + 2], u[0], o);
            for (int i = 0; i < 3; ++i) s[b + i] = o[i];
        }
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) {
            const int b = i + 9 * k;
            axis_inverse(s[b], s[b + 3], s[b + 6], u[1], o);
            for (int j = 0; j < 3; ++j) t[b + 3 * j] = o[j];
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const int b = i + 3 * j;
            axis_inverse(t[b], t[b + 9], t[b + 18], u[2], o);
            for (int k = 0; k < 3; ++k) q[b + 9 * k] = o[k];
        }
}

/* Dense reference: solve sum_a q_a (e_a - u)^m = kappa_m for q with
 * Gaussian elimination (partial pivoting). */
int o3_populations_from_central_solve(const double kappa[27], const double u[3], double q[27]) {
    double A[27][28];
    for (int k = 0; k < 27; ++k) {
        const int mx = k % 3, my = (k / 3) % 3, mz = k / 9;
        for (int a = 0; a < 27; ++a)
            A[k][a] = ipow(ex_of(a) - u[0], mx) * ipow(ey_of(a) - u[1], my) *
                      ipow(ez_of(a) - u[2], mz);
        A[k][27] = kappa[k];
    }
    for (int col = 0; col < 27; ++col) {
        int piv = col;
        for (int r = col + 1; r < 27; ++r)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        if (A[piv][col] == 0.0) return -1;
        if (piv != col)
            for (int c = 0; c < 28; ++c) {
                double tmp = A[col][c];
                A[col][c] = A[piv][c];
                A[piv][c] = tmp;
            }
        for (int r = col + 1; r < 27; ++r) {
            const double f = A[r][col] / A[col][col];
            if (f == 0.0) continue;
            for (int c = col; c < 28; ++c) A[r][c] -= f * A[col][c];
        }
    }
    for (int r = 26; r >= 0; --r) {
        double s = A[r][27];
        for (int c = r + 1; c < 27; ++c) s -= A[r][c] * q[c];
        q[r] = s / A[r][r];
    }
    return 0;
}

/* cs2 powers of the rest state: c(0) = 1, c(1) = 0, c(2) = cs2. */
static double crest(int a) { return a == 0 ? 1.0 : (a == 1 ? 0.0 : CS2); }
/* central moments of a rest distribution about u: m(0) = 1, m(1) = -u,
 * m(2) = cs2 + u^2. */
static double mrest(int a, double u) { return a == 0 ? 1.0 : (a == 1 ? -u : CS2 + u * u); }

void o3_weights(double w[27]) {
    double rest[27];
    for (int k = 0; k < 27; ++k) rest[k] = crest(k % 3) * crest((k / 3) % 3) * crest(k / 9);
    const double zero[3] = {0.0, 0.0, 0.0};
    o3_populations_from_central_solve(rest, zero, w);
}

/* ---------------------------------------------------------------------- */
/* Single-node collisions.                                                */
/* ---------------------------------------------------------------------- */

void o3_collide_scalar(const double q[27], const double u[3], double s, const double j[3],
                       double omega1, double qt[27]) {
    double k[27], kt[27];
    o3_central_moments(q, u, k);
    for (int m = 0; m < 27; ++m) {
        const int mx = m % 3, my = (m / 3) % 3, mz = m / 9;
        double eq = s * crest(mx) * crest(my) * crest(mz);
        double lam = 1.0;
        const int order = mx + my + mz;
        if (order == 1) {
            eq = mx ? j[0] : (my ? j[1] : j[2]);
            lam = omega1;
        }
        kt[m] = k[m] + lam * (eq - k[m]);
    }
    o3_populations_from_central(kt, u, qt);
}

void o3_collide_flow(const double g[27], const double u[3], double P, double rho,
                     const double fp[3], const double ft[3], double omega_zeta, double omega_nu,
                     double gt[27]) {
    double eta[27], eq[27], src[27], th[27];
    o3_central_moments(g, u, eta);
    const double psi = P - rho * CS2;
    const double gam = fp[0] * u[0] + fp[1] * u[1] + fp[2] * u[2];
    for (int m = 0; m < 27; ++m) {
        const int e[3] = {m % 3, (m / 3) % 3, m / 9};
        eq[m] = psi * mrest(e[0], u[0]) * mrest(e[1], u[1]) * mrest(e[2], u[2]) +
                rho * CS2 * crest(e[0]) * crest(e[1]) * crest(e[2]);
        const int order = e[0] + e[1] + e[2];
        src[m] = 0.0;
        if (order == 0) {
            src[m] = gam;
        } else if (order == 1) {
            const int i = e[0] ? 0 : (e[1] ? 1 : 2);
            src[m] = CS2 * ft[i] - u[i] * gam;
        } else if (order == 2) {
            int ax[2], n = 0;
            for (int i = 0; i < 3; ++i)
                for (int r = 0; r < e[i]; ++r) ax[n++] = i;
            const int a = ax[0], b = ax[1];
            if (a == b)
                src[m] = 2.0 * CS2 * fp[a] * u[a] + (u[a] * u[a] + CS2) * gam;
            else
                /* plant 25: the u u gamma term of the off-diagonal source dropped */
                src[m] = CS2 * (fp[a] * u[b] + fp[b] * u[a]) + (PLANT(25) ? 0.0 : u[a] * u[b] * gam);
        }
        /* rate 1 unless second order (below) */
        th[m] = eta[m] + (eq[m] - eta[m]) + 0.5 * src[m];
    }
    /* second order: off-diagonal at omega_nu; diagonal split into the trace
     * (omega_zeta) and the deviatoric parts (omega_nu) */
    const int off[3] = {1 + 3, 1 + 9, 3 + 9};
    for (int r = 0; r < 3; ++r) {
        const int m = off[r];
        th[m] = eta[m] + omega_nu * (eq[m] - eta[m]) + (1.0 - 0.5 * omega_nu) * src[m];
    }
    const int dg[3] = {2, 6, 18};
    double T = 0.0, Te = 0.0, Ts = 0.0;
    for (int r = 0; r < 3; ++r) {
        T += eta[dg[r]];
        Te += eq[dg[r]];
        Ts += src[dg[r]];
    }
    /* plant 23: the trace relaxed at the shear rate */
    const double om_tr = PLANT(23) ? omega_nu : omega_zeta;
    const double Tt = T + om_tr * (Te - T) + (1.0 - 0.5 * om_tr) * Ts;
    for (int r = 0; r < 3; ++r) {
        const int m = dg[r];
        const double d = eta[m] - T / 3.0, de = eq[m] - Te / 3.0, ds = src[m] - Ts / 3.0;
        const double dt = d + omega_nu * (de - d) + (1.0 - 0.5 * omega_nu) * ds;
        th[m] = dt + Tt / 3.0;
    }
    o3_populations_from_central(th, u, gt);
}

/* ---------------------------------------------------------------------- */
/* Whole-grid helpers.                                                    */
/* ---------------------------------------------------------------------- */

static double omega_of(double coeff) { return 1.0 / (coeff / CS2 + 0.5); }

static double lin_phi(const o3_params* p, double phi, double va, double vb) {
    return vb + (phi - p->phi_b) / (p->phi_a - p->phi_b) * (va - vb);
}

#define N3(p) ((size_t)(p)->nx * (size_t)(p)->ny * (size_t)(p)->nz)
#define IDX3(p, x, y, z) (((size_t)(z) * (size_t)(p)->ny + (size_t)(y)) * (size_t)(p)->nx + (size_t)(x))
#define POP3(arr, p, a, x, y, z) ((arr)[(size_t)(a) * N3(p) + IDX3(p, x, y, z)])

static int wrap(int v, int n) {
    v %= n;
    if (v < 0) v += n;
    return v;
}
static int wrap_y(const o3_params* p, int y) {
    const int n = p->ny;
    if (p->walls) {
        while (y < 0 || y >= n) {
            if (y < 0) y = -1 - y;
            if (y >= n) y = 2 * n - 1 - y;
        }
        return y;
    }
    return wrap(y, n);
}

/* Isotropic gradient of a field at node (x, y, z), ghosts as above. */
static void grad3(const o3_params* p, const double* F, const double w[27], int x, int y, int z,
                  double g[3]) {
    double s[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < 27; ++a) {
        const double v =
            F[IDX3(p, wrap(x + ex_of(a), p->nx), wrap_y(p, y + ey_of(a)), wrap(z + ez_of(a), p->nz))];
        s[0] += w[a] * ex_of(a) * v;
        s[1] += w[a] * ey_of(a) * v;
        s[2] += w[a] * ez_of(a) * v;
    }
    /* plant 21: the factor 1/cs2 of the isotropic gradient dropped */
    for (int i = 0; i < 3; ++i) g[i] = PLANT(21) ? s[i] : s[i] / CS2;
}

/* Unit normal arrays with one ghost plane below and above in y (rows -1 and
 * ny), computed from the ghost phi like at any node. */
typedef struct {
    double *phi, *c, *phat, *psih;
    double* nrm[3];
} fields3_t;

#define NIDX(p, x, y, z) (((size_t)(z) * (size_t)((p)->ny + 2) + (size_t)((y) + 1)) * (size_t)(p)->nx + (size_t)(x))

static void fields_alloc3(const o3_params* p, fields3_t* F) {
    const size_t n = N3(p), ne = (size_t)p->nx * (p->ny + 2) * p->nz;
    F->phi = calloc(n, sizeof(double));
    F->c = calloc(n, sizeof(double));
    F->phat = calloc(n, sizeof(double));
    F->psih = calloc(n, sizeof(double));
    for (int i = 0; i < 3; ++i) F->nrm[i] = calloc(ne, sizeof(double));
}
static void fields_free3(fields3_t* F) {
    free(F->phi);
    free(F->c);
    free(F->phat);
    free(F->psih);
    for (int i = 0; i < 3; ++i) free(F->nrm[i]);
}

static void normals3(const o3_params* p, const double w[27], fields3_t* F) {
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = -1; y <= p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                double g[3];
                grad3(p, F->phi, w, x, y, z, g);
                const double mag = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
                for (int i = 0; i < 3; ++i) F->nrm[i][NIDX(p, x, y, z)] = g[i] / (mag + NORMAL_EPS);
            }
}

static void compute_fields3(const o3_params* p, const double w[27], const double* f,
                            const double* h, const double* g, fields3_t* F) {
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                double sf = 0.0, sh = 0.0, sg = 0.0;
                for (int a = 0; a < 27; ++a) {
                    sf += POP3(f, p, a, x, y, z);
                    sh += POP3(h, p, a, x, y, z);
                    if (g) sg += POP3(g, p, a, x, y, z);
                }
                const size_t i = IDX3(p, x, y, z);
                F->phi[i] = sf;
                F->c[i] = sh;
                F->phat[i] = sg;
                F->psih[i] = sg - lin_phi(p, sf, p->rho_a, p->rho_b) * CS2;
            }
    normals3(p, w, F);
}

static double curvature3(const o3_params* p, const fields3_t* F, const double w[27], int x,
                         int y, int z) {
    double s = 0.0;
    for (int a = 0; a < 27; ++a) {
        const int xs = wrap(x + ex_of(a), p->nx), ys = y + ey_of(a), zs = wrap(z + ez_of(a), p->nz);
        const int yy = p->walls ? ys : wrap(ys, p->ny);
        const size_t i = NIDX(p, xs, yy, zs);
        /* plant 26: the corner directions left out of the curvature */
        const int corner = ex_of(a) && ey_of(a) && ez_of(a);
        if (PLANT(26) && corner) continue;
        s += w[a] * (ex_of(a) * F->nrm[0][i] + ey_of(a) * F->nrm[1][i] + ez_of(a) * F->nrm[2][i]);
    }
    return s / CS2;
}

typedef struct {
    double phi, c, P_hat, rho, nu, theta, theta_c, n[3], u[3], P, fp[3], ft[3];
    int fault;
} node3_t;

static double time_factor3(const o3_params* p, int64_t t) {
    return p->vel_period_T == 0.0 ? 1.0 : cos(M_PI * (double)t / p->vel_period_T);
}

static void node_macros3(const o3_params* p, const double w[27], const fields3_t* F,
                         const double* g, const double* ushape, int64_t t, int x, int y, int z,
                         node3_t* s) {
    memset(s, 0, sizeof(*s));
    const size_t i = IDX3(p, x, y, z);
    s->phi = F->phi[i];
    s->c = F->c[i];
    s->P_hat = F->phat[i];
    s->rho = lin_phi(p, s->phi, p->rho_a, p->rho_b);
    s->nu = lin_phi(p, s->phi, p->nu_a, p->nu_b);
    double gphi[3];
    grad3(p, F->phi, w, x, y, z, gphi);
    const double gm2 = gphi[0] * gphi[0] + gphi[1] * gphi[1] + gphi[2] * gphi[2];
    for (int d = 0; d < 3; ++d) s->n[d] = F->nrm[d][NIDX(p, x, y, z)];
    const double dphi = p->phi_a - p->phi_b, phim = 0.5 * (p->phi_a + p->phi_b);
    s->theta = (4.0 / p->W) * (p->phi_a - s->phi) * (s->phi - p->phi_b) / dphi;
    s->theta_c = (8.0 * s->c / p->W) * (phim - s->phi) / dphi;
    if (p->flow == 2) {
        const double curv = curvature3(p, F, w, x, y, z);
        double gc[3], gpsi[3];
        grad3(p, F->c, w, x, y, z, gc);
        grad3(p, F->psih, w, x, y, z, gpsi);
        const double arg = 1.0 - s->c / p->c_max;
        const double sigma = p->sigma0 * (1.0 + p->beta * log(arg));
        if (!(arg > 0.0) || !(sigma >= 0.0)) s->fault |= 2;
        const double dsig = -p->sigma0 * p->beta / (p->c_max - s->c);
        double gs[3], nd = 0.0;
        for (int d = 0; d < 3; ++d) {
            gs[d] = dsig * gc[d];
            nd += s->n[d] * gs[d];
        }
        const double phio = 0.5 * dphi;
        const double ks = 3.0 * p->W / (8.0 * phio * phio);
        const double fext[3] = {p->F_ext_x, p->F_ext_y, p->F_ext_z};
        double j[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 27; ++a) {
            const double v = POP3(g, p, a, x, y, z);
            j[0] += ex_of(a) * v;
            j[1] += ey_of(a) * v;
            j[2] += ez_of(a) * v;
        }
        double gam = 0.0;
        for (int d = 0; d < 3; ++d) {
            const double ts = gs[d] - s->n[d] * nd;
            s->ft[d] = ks * gm2 * (-sigma * curv * s->n[d] + ts) + fext[d];
            s->fp[d] = -gpsi[d];
            s->u[d] = (j[d] + 0.5 * CS2 * s->ft[d]) / (CS2 * s->rho);
            gam += s->fp[d] * s->u[d];
        }
        s->P = s->P_hat + 0.5 * gam;
    } else if (p->flow == 1) {
        const double tf = time_factor3(p, t);
        for (int d = 0; d < 3; ++d) s->u[d] = ushape[(size_t)d * N3(p) + i] * tf;
    }
    if (!isfinite(s->phi) || !isfinite(s->c) || !isfinite(s->u[0]) || !isfinite(s->u[1]) ||
        !isfinite(s->u[2]) || !isfinite(s->P))
        s->fault |= 1;
}

int o3_check_params(const o3_params* p) {
    if (p->nx < 4 || p->ny < 4 || p->nz < 1) return -1;
    if (!(p->phi_a != p->phi_b) || !(p->W > 0.0)) return -1;
    const double wk = omega_of(p->M_phi), wc = omega_of(p->D_s);
    if (!(wk > 0.0 && wk < 2.0) || !(wc > 0.0 && wc < 2.0)) return -2;
    if (p->flow == 2) {
        const double w1 = omega_of(p->nu_a), w2 = omega_of(p->nu_b);
        if (!(w1 > 0.0 && w1 < 2.0) || !(w2 > 0.0 && w2 < 2.0)) return -2;
        if (!(p->omega_zeta > 0.0 && p->omega_zeta < 2.0)) return -2;
        if (!(p->rho_a > 0.0 && p->rho_b > 0.0) || !(p->c_max > 0.0)) return -1;
    }
    return 0;
}

int o3_init(const o3_params* p, const double* phi, const double* c, const double* ux,
            const double* uy, const double* uz, const double* P, double* f, double* h,
            double* g) {
    if (o3_check_params(p) != 0) return -1;
    double w[27];
    o3_weights(w);
    fields3_t F;
    fields_alloc3(p, &F);
    memcpy(F.phi, phi, sizeof(double) * N3(p));
    normals3(p, w, &F);
    const double dphi = p->phi_a - p->phi_b, phim = 0.5 * (p->phi_a + p->phi_b);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                const size_t i = IDX3(p, x, y, z);
                const double u[3] = {ux ? ux[i] : 0.0, uy ? uy[i] : 0.0, uz ? uz[i] : 0.0};
                const double ph = phi[i], cc = c[i];
                double n[3];
                for (int d = 0; d < 3; ++d) n[d] = F.nrm[d][NIDX(p, x, y, z)];
                const double theta = (4.0 / p->W) * (p->phi_a - ph) * (ph - p->phi_b) / dphi;
                const double theta_c = (8.0 * cc / p->W) * (phim - ph) / dphi;
                double kf[27], kh[27], qf[27], qh[27];
                for (int m = 0; m < 27; ++m) {
                    const int mx = m % 3, my = (m / 3) % 3, mz = m / 9;
                    const double r = crest(mx) * crest(my) * crest(mz);
                    kf[m] = ph * r;
                    kh[m] = cc * r;
                    if (mx + my + mz == 1) {
                        const int d = mx ? 0 : (my ? 1 : 2);
                        kf[m] = p->M_phi * theta * n[d];
                        kh[m] = p->D_s * theta_c * n[d];
                    }
                }
                o3_populations_from_central(kf, u, qf);
                o3_populations_from_central(kh, u, qh);
                for (int a = 0; a < 27; ++a) {
                    POP3(f, p, a, x, y, z) = qf[a];
                    POP3(h, p, a, x, y, z) = qh[a];
                }
                if (p->flow == 2 && g) {
                    const double rho = lin_phi(p, ph, p->rho_a, p->rho_b);
                    const double Pv = P ? P[i] : rho * CS2;
                    const double psi = Pv - rho * CS2;
                    double eq[27], qg[27];
                    for (int m = 0; m < 27; ++m) {
                        const int e0 = m % 3, e1 = (m / 3) % 3, e2 = m / 9;
                        eq[m] = psi * mrest(e0, u[0]) * mrest(e1, u[1]) * mrest(e2, u[2]) +
                                rho * CS2 * crest(e0) * crest(e1) * crest(e2);
                    }
                    o3_populations_from_central(eq, u, qg);
                    for (int a = 0; a < 27; ++a) POP3(g, p, a, x, y, z) = qg[a];
                }
            }
    fields_free3(&F);
    return 0;
}

int o3_step(const o3_params* p, int64_t t, const double* ushape, const double* f,
            const double* h, const double* g, double* f2, double* h2, double* g2) {
    if (o3_check_params(p) != 0) return -1;
    double w[27];
    o3_weights(w);
    const int coupled = p->flow == 2;
    fields3_t F;
    fields_alloc3(p, &F);
    compute_fields3(p, w, f, h, coupled ? g : NULL, &F);
    const double omega_k = omega_of(p->M_phi), omega_c = omega_of(p->D_s);
    int fault = 0;
#pragma omp parallel for schedule(static) reduction(| : fault)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                node3_t s;
                node_macros3(p, w, &F, g, ushape, t, x, y, z, &s);
                fault |= s.fault;
                double qf[27], qh[27], qg[27], tf[27], th[27], tg[27];
                for (int a = 0; a < 27; ++a) {
                    qf[a] = POP3(f, p, a, x, y, z);
                    qh[a] = POP3(h, p, a, x, y, z);
                }
                double jf[3], jh[3];
                for (int d = 0; d < 3; ++d) {
                    jf[d] = p->M_phi * s.theta * s.n[d];
                    jh[d] = p->D_s * s.theta_c * s.n[d];
                }
                o3_collide_scalar(qf, s.u, s.phi, jf, omega_k, tf);
                o3_collide_scalar(qh, s.u, s.c, jh, omega_c, th);
                if (coupled) {
                    for (int a = 0; a < 27; ++a) qg[a] = POP3(g, p, a, x, y, z);
                    o3_collide_flow(qg, s.u, s.P, s.rho, s.fp, s.ft, p->omega_zeta, omega_of(s.nu),
                                    tg);
                }
                for (int a = 0; a < 27; ++a) {
                    /* plant 24: streamed against the direction along z */
                    int xd = wrap(x + ex_of(a), p->nx), yd = y + ey_of(a),
                        zd = wrap(z + (PLANT(24) ? -ez_of(a) : ez_of(a)), p->nz);
                    int ad = a;
                    double corr = 0.0;
                    if (p->walls && (yd < 0 || yd >= p->ny)) {
                        /* half-way bounce-back into the opposite direction */
                        ad = opposite(a);
                        xd = x;
                        zd = z;
                        const double uw = yd < 0 ? -p->u_wall : p->u_wall;
                        corr = 2.0 * w[ad] * s.rho * (ex_of(ad) * uw);
                        yd = y;
                    } else {
                        yd = wrap_y(p, yd);
                    }
                    POP3(f2, p, ad, xd, yd, zd) = tf[a];
                    POP3(h2, p, ad, xd, yd, zd) = th[a];
                    if (coupled) POP3(g2, p, ad, xd, yd, zd) = tg[a] + corr;
                }
            }
    fields_free3(&F);
    return fault;
}

int o3_run(const o3_params* p, int64_t t0, int64_t nsteps, const double* ushape, double* f,
           double* h, double* g) {
    const size_t n = (size_t)27 * N3(p);
    double* f2 = malloc(n * sizeof(double));
    double* h2 = malloc(n * sizeof(double));
    double* g2 = g ? malloc(n * sizeof(double)) : NULL;
    int fault = 0;
    for (int64_t s = 0; s < nsteps; ++s) {
        fault |= o3_step(p, t0 + s, ushape, f, h, g, f2, h2, g2);
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

int o3_fields(const o3_params* p, int64_t t, const double* ushape, const double* f,
              const double* h, const double* g, double* phi, double* c, double* ux,
              double* uy, double* uz, double* P) {
    double w[27];
    o3_weights(w);
    const int coupled = p->flow == 2;
    fields3_t F;
    fields_alloc3(p, &F);
    compute_fields3(p, w, f, h, coupled ? g : NULL, &F);
    int fault = 0;
#pragma omp parallel for schedule(static) reduction(| : fault)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                node3_t s;
                node_macros3(p, w, &F, g, ushape, t, x, y, z, &s);
                fault |= s.fault;
                const size_t i = IDX3(p, x, y, z);
                if (phi) phi[i] = s.phi;
                if (c) c[i] = s.c;
                if (ux) ux[i] = s.u[0];
                if (uy) uy[i] = s.u[1];
                if (uz) uz[i] = s.u[2];
                if (P) P[i] = s.P;
            }
    fields_free3(&F);
    return fault;
}
