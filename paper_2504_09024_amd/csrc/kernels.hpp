// HIP kernels of the coupled central-moment LB step (arXiv 2504.09024) for
// gfx950.  One fused kernel performs a whole time step for every tile of
// every simulation in the context:
//
//   phase 1  load the 27 (18 without flow) pre-collision populations of the
//            tile's own nodes into registers; zeroth moments phi, c and the
//            pressure deviation P^ - P_ref go to LDS; the halo ring
//            (radius 2 for phi, radius 1 for c and P^) is summed from the
//            neighbours' populations;
//   phase 2  unit normal n = grad phi/(|grad phi| + eps) on the radius-1
//            ring (coupled flow only, it feeds the curvature);
//   phase 3  per node: interface geometry (theta, theta_c, curvature),
//            Langmuir sigma(c), F_s, F_p, u, P; central-moment collisions
//            of f, h and g; push-streaming of the post-collision
//            populations to the neighbours (half-way bounce-back at walls).
//
// The population state between steps is the pre-collision state at each
// node (push form), so the zeroth moments of any node are local sums.
#pragma once
#include "lattice.hpp"

namespace cmlb {

constexpr int TX = 64;          // tile width: one wavefront across x
constexpr int WG = 256;         // threads per workgroup (4 waves)
constexpr double NORMAL_EPS = 1e-12;

struct StepArgs {
    const void* src;
    void* dst;
    const SimDev* sims;
    const int4* tiles;      // (sim, x0, y0, -)
    int32_t tile_base;
    int32_t pad_;
    const void* ushape;     // prescribed velocity shapes, compute type
    const int64_t* step_in; // step counter read by this launch
    int64_t* step_out;      // step counter written (n + 1) by workgroup 0
    int32_t* fault;         // per-sim fault bits
    double* fields_out;     // fields mode: [5][ny][nx] (phi, c, ux, uy, P)
};

template <class S>
struct Store {
    static constexpr bool scaled = false;
};
template <>
struct Store<_Float16> {
    static constexpr bool scaled = true;
};

// Load the nine stored values of a scalar lattice (q_a/w_a - qref, scaled).
template <class S, class T>
__device__ __forceinline__ void load9(const S* __restrict__ p, int plane, T v[9]) {
#pragma unroll
    for (int a = 0; a < 9; ++a) v[a] = T(p[a * plane]);
}

// Moments of stored scalar-lattice values in storage units.  No FP
// contraction: a node's zeroth moment must carry the same bits in every code
// path that computes it (tile interior and neighbouring tiles' halos).
template <class T>
__device__ __forceinline__ void scalar_moments_nc(const T v[9], T& m0, T& m1, T& m2) {
#pragma clang fp contract(off)
    scalar_moments(v, m0, m1, m2);
}
template <class T>
__device__ __forceinline__ T scalar_zeroth_nc(const T v[9]) {
#pragma clang fp contract(off)
    T m0, m1, m2;
    scalar_moments(v, m0, m1, m2);
    return m0;
}

// Decode nine stored values of g to deviations d_a = w_a s_a inv.
template <class S, class T>
__device__ __forceinline__ void decode_dev(const S* __restrict__ p, int plane, T inv, T d[9]) {
#pragma clang fp contract(off)
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const T s = T(p[a * plane]);
        if (Store<S>::scaled)
            d[a] = wgt<T>(a) * (s * inv);
        else
            d[a] = wgt<T>(a) * s;
    }
}

template <class T>
__device__ __forceinline__ T zeroth(const T d[9]) {
#pragma clang fp contract(off)
    return sum9(d);
}

template <class T>
__device__ __forceinline__ Raw6<T> moments6_nc(const T d[9]) {
#pragma clang fp contract(off)
    return raw_moments6(d);
}

template <class T>
struct Consts {
    T inv_f, qref_f, inv_h, inv_g;
    T scale_f, scale_h, scale_g;
    T phi_a, phi_b, inv_dphi, phim, theta_k, thetac_k;
    T M_phi, D_s, omega_k, omega_c;
    T rho_b, drho, nu_b, dnu, omega_zeta;
    T sigma0, beta, c_max, ks;
    T u_wall, Fx, Fy, P_ref;
};

template <class T>
__device__ __forceinline__ Consts<T> load_consts(const SimDev* sd) {
    Consts<T> k;
    k.scale_f = T(sd->scale_f);
    k.scale_h = T(sd->scale_h);
    k.scale_g = T(sd->scale_g);
    k.inv_f = T(1.0 / sd->scale_f);
    k.inv_h = T(1.0 / sd->scale_h);
    k.inv_g = T(1.0 / sd->scale_g);
    k.qref_f = T(sd->qref_f);
    k.phi_a = T(sd->phi_a);
    k.phi_b = T(sd->phi_b);
    k.inv_dphi = T(sd->inv_dphi);
    k.phim = T(sd->phim);
    k.theta_k = T(sd->theta_k);
    k.thetac_k = T(sd->thetac_k);
    k.M_phi = T(sd->M_phi);
    k.D_s = T(sd->D_s);
    k.omega_k = T(sd->omega_k);
    k.omega_c = T(sd->omega_c);
    k.rho_b = T(sd->rho_b);
    k.drho = T(sd->drho);
    k.nu_b = T(sd->nu_b);
    k.dnu = T(sd->dnu);
    k.omega_zeta = T(sd->omega_zeta);
    k.sigma0 = T(sd->sigma0);
    k.beta = T(sd->beta);
    k.c_max = T(sd->c_max);
    k.ks = T(sd->ks);
    k.u_wall = T(sd->u_wall);
    k.Fx = T(sd->F_ext_x);
    k.Fy = T(sd->F_ext_y);
    k.P_ref = T(sd->P_ref);
    return k;
}

// ---------------------------------------------------------------------------
// The fused step kernel.  FIELDS = true evaluates phases 1-3 up to the
// macroscopic fields and writes them instead of colliding.
// ---------------------------------------------------------------------------
template <class S, class T, int FLOW, bool WALLS, int NPT, bool FIELDS>
__global__ __launch_bounds__(WG) void k_step(const StepArgs a) {
    constexpr bool CPL = FLOW == FLOW_COUPLED;
    constexpr bool MOV = FLOW != FLOW_NONE;
    constexpr int NL = CPL ? 3 : 2;
    constexpr int TY = 4 * NPT;
    constexpr int PW = TX + 4, PH = TY + 4;  // phi region (radius 2)
    constexpr int QW = TX + 2, QH = TY + 2;  // c, P^, n region (radius 1)
    constexpr int RING = 4 * PW + 4 * TY;
    __shared__ T phiL[PH * PW];
    __shared__ T cL[QH * QW];
    __shared__ T pL[CPL ? QH * QW : 1];
    __shared__ T nxL[CPL ? QH * QW : 1];
    __shared__ T nyL[CPL ? QH * QW : 1];

    const int4 tl = a.tiles[a.tile_base + blockIdx.x];
    const SimDev* sd = a.sims + tl.x;
    const int nx = sd->nx, ny = sd->ny;
    const int x0 = tl.y, y0 = tl.z;
    const int plane = nx * ny;
    const S* __restrict__ src = static_cast<const S*>(a.src) + sd->off;
    const Consts<T> k = load_consts<T>(sd);
    const int64_t step = *a.step_in;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int gx = x0 + lane;
    const int lx = wrap_coord(gx, nx);

    // ---------------- phase 1: own nodes -----------------------------------
    T qf[NPT][9], qh[NPT][9], qg[CPL ? NPT : 1][9];
    T phv[NPT], cv[NPT], phn[NPT], chn[NPT], jfx[NPT], jfy[NPT], jhx[NPT], jhy[NPT];
    Raw6<T> mg[CPL ? NPT : 1];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int iy = wave * NPT + j;
        const int gy = y0 + iy;
        const int ly = WALLS ? mirror_coord(gy, ny) : wrap_coord(gy, ny);
        const int nidx = ly * nx + lx;
        load9<S, T>(src + nidx, plane, qf[j]);
        load9<S, T>(src + 9 * plane + nidx, plane, qh[j]);
        scalar_moments_nc(qf[j], phn[j], jfx[j], jfy[j]);
        scalar_moments_nc(qh[j], chn[j], jhx[j], jhy[j]);
        // true zeroth and first moments
        phv[j] = phn[j] * k.inv_f + k.qref_f;
        cv[j] = chn[j] * k.inv_h;
        jfx[j] *= k.inv_f;
        jfy[j] *= k.inv_f;
        jhx[j] *= k.inv_h;
        jhy[j] *= k.inv_h;
        phiL[(iy + 2) * PW + lane + 2] = phv[j];
        cL[(iy + 1) * QW + lane + 1] = cv[j];
        if constexpr (CPL) {
            decode_dev<S, T>(src + 18 * plane + nidx, plane, k.inv_g, qg[j]);
            mg[j] = moments6_nc(qg[j]);
            pL[(iy + 1) * QW + lane + 1] = mg[j].m0;
        }
    }
    // ---------------- phase 1b: halo ring ----------------------------------
    for (int i = tid; i < RING; i += WG) {
        int ry, rx;
        if (i < 2 * PW) {
            ry = i / PW;
            rx = i - ry * PW;
        } else if (i < 4 * PW) {
            const int j = i - 2 * PW;
            const int r = j / PW;
            ry = PH - 2 + r;
            rx = j - r * PW;
        } else {
            int j = i - 4 * PW;
            const int side = j / (2 * TY);
            j -= side * 2 * TY;
            ry = 2 + (j >> 1);
            rx = (j & 1) + side * (PW - 2);
        }
        const int hx = wrap_coord(x0 - 2 + rx, nx);
        const int hy = WALLS ? mirror_coord(y0 - 2 + ry, ny) : wrap_coord(y0 - 2 + ry, ny);
        const int nidx = hy * nx + hx;
        T q[9];
        load9<S, T>(src + nidx, plane, q);
        phiL[ry * PW + rx] = scalar_zeroth_nc(q) * k.inv_f + k.qref_f;
        if (ry >= 1 && ry <= PH - 2 && rx >= 1 && rx <= PW - 2) {
            const int qi = (ry - 1) * QW + rx - 1;
            load9<S, T>(src + 9 * plane + nidx, plane, q);
            cL[qi] = scalar_zeroth_nc(q) * k.inv_h;
            if constexpr (CPL) {
                decode_dev<S, T>(src + 18 * plane + nidx, plane, k.inv_g, q);
                pL[qi] = zeroth(q);
            }
        }
    }
    __syncthreads();

    // ---------------- phase 2: unit normal on the radius-1 region ----------
    if constexpr (CPL) {
        for (int i = tid; i < QH * QW; i += WG) {
            const int qy = i / QW, qx = i - qy * QW;
            T gxv, gyv;
            lds_grad<T, PW>(phiL, (qy + 1) * PW + qx + 1, gxv, gyv);
            const T inv = T(1) / (sqrt(gxv * gxv + gyv * gyv) + T(NORMAL_EPS));
            nxL[i] = gxv * inv;
            nyL[i] = gyv * inv;
        }
        __syncthreads();
    }

    // ---------------- phase 3: per-node physics, collision, streaming ------
    T tf = T(1);
    if constexpr (FLOW == FLOW_PRESCRIBED) {
        if (sd->vel_period_T != 0.0) tf = T(cos(M_PI * (double)step / sd->vel_period_T));
    }
    S* __restrict__ dst = static_cast<S*>(a.dst) + sd->off;
    int fault = 0;
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int iy = wave * NPT + j;
        const int gy = y0 + iy;
        const bool valid = gx < nx && gy < ny;
        const int pidx = (iy + 2) * PW + lane + 2;
        const int qidx = (iy + 1) * QW + lane + 1;
        const T phi = phv[j], c = cv[j];
        T gpx, gpy;
        lds_grad<T, PW>(phiL, pidx, gpx, gpy);
        const T gm2 = gpx * gpx + gpy * gpy;
        T nxv, nyv;
        if constexpr (CPL) {
            nxv = nxL[qidx];
            nyv = nyL[qidx];
        } else {
            const T inv = T(1) / (sqrt(gm2) + T(NORMAL_EPS));
            nxv = gpx * inv;
            nyv = gpy * inv;
        }
        const T theta = k.theta_k * (k.phi_a - phi) * (phi - k.phi_b) * k.inv_dphi;
        const T theta_c = k.thetac_k * c * (k.phim - phi) * k.inv_dphi;

        T ux = T(0), uy = T(0), dP = T(0), rho = T(1), psi = T(0);
        T fpx = T(0), fpy = T(0), ftx = T(0), fty = T(0), gam = T(0), omega_nu = T(1);
        if constexpr (CPL) {
            T dnx_dx, dnx_dy, dny_dx, dny_dy, gcx, gcy, gqx, gqy;
            lds_grad<T, QW>(nxL, qidx, dnx_dx, dnx_dy);
            lds_grad<T, QW>(nyL, qidx, dny_dx, dny_dy);
            lds_grad<T, QW>(cL, qidx, gcx, gcy);
            lds_grad<T, QW>(pL, qidx, gqx, gqy);
            const T curv = dnx_dx + dny_dy;
            const T lam = (phi - k.phi_b) * k.inv_dphi;
            rho = k.rho_b + lam * k.drho;
            const T nu = k.nu_b + lam * k.dnu;
            omega_nu = T(1) / (T(3) * nu + T(0.5));
            const T arg = T(1) - c / k.c_max;
            const T sigma = k.sigma0 * (T(1) + k.beta * log(arg));
            if (valid && (!(arg > T(0)) || !(sigma >= T(0)))) fault |= 2;
            const T dsig = -k.sigma0 * k.beta / (k.c_max - c);
            const T gsx = dsig * gcx, gsy = dsig * gcy;
            const T nd = nxv * gsx + nyv * gsy;
            const T tsx = gsx - nxv * nd, tsy = gsy - nyv * nd;
            const T wk = k.ks * gm2;
            ftx = wk * (tsx - sigma * curv * nxv) + k.Fx;
            fty = wk * (tsy - sigma * curv * nyv) + k.Fy;
            // F_p = -grad psi^, psi^ = P^ - rho cs2, rho linear in phi
            const T dr = k.drho * k.inv_dphi * K<T>::cs2;
            fpx = -(gqx - dr * gpx);
            fpy = -(gqy - dr * gpy);
            const T inv_rho = T(1) / rho;
            ux = (T(3) * mg[j].m1 + T(0.5) * ftx) * inv_rho;
            uy = (T(3) * mg[j].m2 + T(0.5) * fty) * inv_rho;
            gam = fpx * ux + fpy * uy;
            dP = mg[j].m0 + T(0.5) * gam;
            psi = dP + (k.P_ref - rho * K<T>::cs2);
        } else if constexpr (FLOW == FLOW_PRESCRIBED) {
            const T* us = static_cast<const T*>(a.ushape) + sd->ushape_off;
            const int ni = gy < ny ? gy * nx + lx : lx;
            ux = us[ni] * tf;
            uy = us[plane + ni] * tf;
        }
        if (valid && !(isfinite(phi) && isfinite(c) && isfinite(ux) && isfinite(uy) &&
                       isfinite(dP)))
            fault |= 1;

        if constexpr (FIELDS) {
            if (valid) {
                double* o = a.fields_out;
                const int i = gy * nx + gx;
                o[i] = double(phi);
                o[plane + i] = double(c);
                o[2 * plane + i] = double(ux);
                o[3 * plane + i] = double(uy);
                o[4 * plane + i] = CPL ? double(k.P_ref) + double(dP) : 0.0;
            }
            continue;
        } else {
            // f: phase field (App. C).  Stored result = the node's own zeroth
            // moment (storage units) + P^-1 of the raw-moment deviation.
            T r[9], s[9];
            {
                const T k1 = (T(1) - k.omega_k) * (jfx[j] - ux * phi) + k.omega_k * k.M_phi * theta * nxv;
                const T k2 = (T(1) - k.omega_k) * (jfy[j] - uy * phi) + k.omega_k * k.M_phi * theta * nyv;
                scalar_post_dev<T, MOV>(phi, k1, k2, ux, uy, r);
                pinv_dev(r, k.scale_f, s);
#pragma unroll
                for (int q = 0; q < 9; ++q) qf[j][q] = phn[j] + s[q];
            }
            // h: interface-bound surfactant (Sec. 3)
            {
                const T k1 = (T(1) - k.omega_c) * (jhx[j] - ux * c) + k.omega_c * k.D_s * theta_c * nxv;
                const T k2 = (T(1) - k.omega_c) * (jhy[j] - uy * c) + k.omega_c * k.D_s * theta_c * nyv;
                scalar_post_dev<T, MOV>(c, k1, k2, ux, uy, r);
                pinv_dev(r, k.scale_h, s);
#pragma unroll
                for (int q = 0; q < 9; ++q) qh[j][q] = chn[j] + s[q];
            }
            // g: two-fluid flow (App. D)
            if constexpr (CPL) {
                T t[9];
                const T P_hat = k.P_ref + mg[j].m0;
                flow_collide(mg[j], ux, uy, dP, psi, P_hat, fpx, fpy, ftx, fty, gam,
                             k.omega_zeta, omega_nu, t);
                flow_post_raw(t, ux, uy, k.P_ref, r);
                pinv_encode(r, k.scale_g, T(0), s);
#pragma unroll
                for (int q = 0; q < 9; ++q) qg[j][q] = s[q];
            }
            if (valid) {
                const T corr = T(2) * rho * k.u_wall * k.scale_g;  // 2 rho |u_w| scale
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    const int ex = EXa(q), ey = EYa(q);
                    int dx = gx + ex, dy = gy + ey;
                    int dq = q;
                    T cg = T(0);
                    if (WALLS && (dy < 0 || dy >= ny)) {
                        dq = OPPa(q);
                        dx = gx;
                        // e_opp . u_w with u_w = -u_wall below, +u_wall above
                        const int exo = EXa(dq);
                        cg = (dy < 0 ? -corr : corr) * T(exo);
                        dy = gy;
                    } else {
                        if (dx >= nx) dx -= nx;
                        if (dx < 0) dx += nx;
                        if (!WALLS) {
                            if (dy >= ny) dy -= ny;
                            if (dy < 0) dy += ny;
                        }
                    }
                    const int o = dq * plane + dy * nx + dx;
                    dst[o] = S(qf[j][q]);
                    dst[9 * plane + o] = S(qh[j][q]);
                    if constexpr (CPL) dst[18 * plane + o] = S(qg[j][q] + cg);
                }
            }
        }
    }
    (void)NL;
    if (fault) atomicOr(a.fault + tl.x, fault);
    if constexpr (!FIELDS) {
        if (blockIdx.x == 0 && tid == 0) *a.step_out = step + 1;
    }
}

// ---------------------------------------------------------------------------
// Initialisation: populations at the central-moment equilibria of given
// fields (computed in FP64, encoded to the storage precision).
// ---------------------------------------------------------------------------
struct InitArgs {
    void* pop;               // sim's population block
    const SimDev* sd;
    const double* phi;
    const double* c;
    const double* ux;        // may be null
    const double* uy;        // may be null
    const double* P;         // may be null
    void* ushape;            // prescribed shapes (compute type), may be null
    int32_t flow, walls;
};

template <class S, class T>
__global__ __launch_bounds__(WG) void k_init(const InitArgs a) {
    const SimDev* sd = a.sd;
    const int nx = sd->nx, ny = sd->ny, plane = nx * ny;
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i >= plane) return;
    const int x = i % nx, y = i / nx;
    // isotropic gradient of phi with the ghost rules of the step kernel
    double gxv = 0.0, gyv = 0.0;
    {
        auto at = [&](int dx, int dy) {
            const int xx = wrap_coord(x + dx, nx);
            const int yy = a.walls ? mirror_coord(y + dy, ny) : wrap_coord(y + dy, ny);
            return a.phi[yy * nx + xx];
        };
        const double e = at(1, 0), w = at(-1, 0), n = at(0, 1), s = at(0, -1);
        const double ne = at(1, 1), nw = at(-1, 1), se = at(1, -1), sw = at(-1, -1);
        gxv = (e - w) * K<double>::third + ((ne - nw) + (se - sw)) * K<double>::twelfth;
        gyv = (n - s) * K<double>::third + ((ne + nw) - (se + sw)) * K<double>::twelfth;
    }
    const double inv = 1.0 / (sqrt(gxv * gxv + gyv * gyv) + NORMAL_EPS);
    const double nxv = gxv * inv, nyv = gyv * inv;
    const double phi = a.phi[i], c = a.c[i];
    const double ux = a.ux ? a.ux[i] : 0.0, uy = a.uy ? a.uy[i] : 0.0;
    const double theta = sd->theta_k * (sd->phi_a - phi) * (phi - sd->phi_b) * sd->inv_dphi;
    const double theta_c = sd->thetac_k * c * (sd->phim - phi) * sd->inv_dphi;
    S* pop = static_cast<S*>(a.pop);
    double r[9], s[9];
    scalar_post_dev<double, true>(phi, sd->M_phi * theta * nxv, sd->M_phi * theta * nyv, ux, uy, r);
    pinv_dev(r, sd->scale_f, s);
    const double phin = (phi - sd->qref_f) * sd->scale_f;
    for (int q = 0; q < 9; ++q) pop[q * plane + i] = S(phin + s[q]);
    scalar_post_dev<double, true>(c, sd->D_s * theta_c * nxv, sd->D_s * theta_c * nyv, ux, uy, r);
    pinv_dev(r, sd->scale_h, s);
    const double chn = c * sd->scale_h;
    for (int q = 0; q < 9; ++q) pop[(9 + q) * plane + i] = S(chn + s[q]);
    if (a.flow == FLOW_COUPLED) {
        const double lam = (phi - sd->phi_b) * sd->inv_dphi;
        const double rho = sd->rho_b + lam * sd->drho;
        const double P = a.P ? a.P[i] : rho * K<double>::cs2;
        const double psi = P - rho * K<double>::cs2;
        double t[9];
        flow_eq_dev(P - sd->P_ref, psi, ux, uy, t);
        flow_post_raw(t, ux, uy, sd->P_ref, r);
        pinv_encode(r, sd->scale_g, 0.0, s);
        for (int q = 0; q < 9; ++q) pop[(18 + q) * plane + i] = S(s[q]);
    }
    if (a.flow == FLOW_PRESCRIBED && a.ushape) {
        T* us = static_cast<T*>(a.ushape);
        us[i] = T(ux);
        us[plane + i] = T(uy);
    }
}

// ---------------------------------------------------------------------------
// Population transfer: decode to / encode from plain FP64 populations.
// ---------------------------------------------------------------------------
template <class S>
__global__ __launch_bounds__(WG) void k_decode(const void* pop, const SimDev* sd, int nlat,
                                               double* out) {
    const int plane = sd->nx * sd->ny;
    const int64_t total = (int64_t)nlat * 9 * plane;
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= total) return;
    const int lat = (int)(i / (9 * (int64_t)plane));
    const int q = (int)((i / plane) % 9);
    const double s = double(static_cast<const S*>(pop)[i]);
    const double w = wgt<double>(q);
    const double scale = lat == 0 ? sd->scale_f : (lat == 1 ? sd->scale_h : sd->scale_g);
    const double qref = lat == 0 ? sd->qref_f : (lat == 1 ? 0.0 : sd->P_ref);
    out[i] = w * (s / scale + qref);
}

template <class S>
__global__ __launch_bounds__(WG) void k_encode(void* pop, const SimDev* sd, int nlat,
                                               const double* in) {
    const int plane = sd->nx * sd->ny;
    const int64_t total = (int64_t)nlat * 9 * plane;
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= total) return;
    const int lat = (int)(i / (9 * (int64_t)plane));
    const int q = (int)((i / plane) % 9);
    const double scale = lat == 0 ? sd->scale_f : (lat == 1 ? sd->scale_h : sd->scale_g);
    const double qref = lat == 0 ? sd->qref_f : (lat == 1 ? 0.0 : sd->P_ref);
    const double s = (in[i] * inv_wgt<double>(q) - qref) * scale;
    static_cast<S*>(pop)[i] = S(s);
}

// ---------------------------------------------------------------------------
// Inventories: FP64 totals of phi and c.  One workgroup per row; each
// thread sums its columns in order, then a fixed butterfly over the wave
// and a fixed order over the waves; a second kernel sums the rows in order.
// The result does not depend on the step kernel's tiling.
// ---------------------------------------------------------------------------
template <class S>
__global__ __launch_bounds__(WG) void k_inventory_rows(const void* pop, const SimDev* sd,
                                                       double* rows) {
    const int nx = sd->nx, ny = sd->ny, plane = nx * ny;
    const int y = blockIdx.x;
    const S* p = static_cast<const S*>(pop);
    const double inv_f = 1.0 / sd->scale_f, inv_h = 1.0 / sd->scale_h, qref = sd->qref_f;
    double sf = 0.0, sh = 0.0;
    for (int x = threadIdx.x; x < nx; x += WG) {
        const int i = y * nx + x;
        double vf = 0.0, vh = 0.0;
        for (int q = 0; q < 9; ++q) {
            const double w = wgt<double>(q);
            vf += w * (double(p[q * plane + i]) * inv_f + qref);
            vh += w * (double(p[(9 + q) * plane + i]) * inv_h);
        }
        sf += vf;
        sh += vh;
    }
    for (int m = 32; m >= 1; m >>= 1) {
        sf += __shfl_xor(sf, m);
        sh += __shfl_xor(sh, m);
    }
    __shared__ double red[2][WG / 64];
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = sf;
        red[1][threadIdx.x >> 6] = sh;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < WG / 64; ++w) {
            a += red[0][w];
            b += red[1][w];
        }
        rows[2 * y] = a;
        rows[2 * y + 1] = b;
    }
}

__global__ void k_inventory_final(const double* rows, int ny, double* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0.0, b = 0.0;
    for (int y = 0; y < ny; ++y) {
        a += rows[2 * y];
        b += rows[2 * y + 1];
    }
    out[0] = a;
    out[1] = b;
}

}  // namespace cmlb
