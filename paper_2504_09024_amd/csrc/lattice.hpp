// Device-side arithmetic of the coupled central-moment LB step on gfx950.
//
// Notation follows arXiv 2504.09024: f (phase field phi, App. C), h
// (interface-bound surfactant c, Sec. 3), g (pressure-based flow P, u,
// App. D).  D2Q9 directions (Eqs. ex/ey, e_8 = (+1, -1)):
//     a :  0  1  2  3  4  5  6  7  8
//    ex :  0  1  0 -1  0  1 -1 -1  1
//    ey :  0  0  1  0 -1  1  1 -1 -1
// rest weights w = 4/9, 1/9 (a = 1..4), 1/36 (a = 5..8): the populations
// whose raw moments are those of the rest state (1,0,0,cs2,cs2,0,0,0,cs2^2).
//
// Storage.  Population a of lattice L is held as
//     s_a = (q_a / w_a - qref_L) * scale_L
// i.e. the deviation from the rest equilibrium w_a qref_L divided by w_a.
// For g, qref = P_ref = rho_b cs2 and all collision arithmetic is done in
// deviation form (every O(1) rest contribution is removed analytically), so
// FP32 arithmetic keeps ~1e-7 relative accuracy on u ~ 1e-4.  For f and h
// the arithmetic uses the true populations (their values are O(phi), O(c)).
//
// Collision closed forms.  Because the relaxation matrices of App. C and
// Sec. 3 are diag(1, w1, w1, 1, ..., 1), the post-collision central moments
// of f and h are (s, k1, k2, cs2 s, cs2 s, 0, 0, 0, cs2^2 s) with
// k1 = (1 - w1) kappa_10 + w1 J_x: only the first-order central moments of
// the input survive.  For g (App. D) only eta_20, eta_02 and eta_11 survive
// (rates omega_zeta on the trace, omega_nu on the deviator and eta_11).
// The back-transform applies F^-1(u) of App. B (rows 6-8 from the binomial
// expansion of the central-moment definition) and P^-1 of App. A.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"

namespace cmlb {

enum { FLOW_NONE = 0, FLOW_PRESCRIBED = 1, FLOW_COUPLED = 2 };

// Physical and storage constants of one simulation in the compute type, so
// kernels read them with scalar loads and never convert on the device.
template <class T>
struct PhysConsts {
    T inv_f, qref_f, inv_h, inv_g;    // storage decode: 1/scale, phi reference
    T wdec0, wdec1, wdec5;            // w_a / scale_g for a = 0, 1..4, 5..8 (scaled g)
    T scale_f, scale_h, scale_g;      // storage encode scales (powers of two)
    T phi_a, phi_b, inv_dphi, phim;   // phase bounds, 1/(phi_a - phi_b), midpoint
    T theta_k, thetac_k;              // 4/W and 8/W
    T M_phi, D_s, omega_k, omega_c;   // mobility, diffusivity and their rates
    T rho_b, drho, nu_b, dnu;         // rho, nu linear in phi
    T inv_rho_b, omega_nu_b;          // used when drho == 0 / dnu == 0
    T omega_zeta;
    T sigma0, beta, c_max, inv_cmax, ks;  // Langmuir isotherm, F_s normalisation
    T u_wall, Fx, Fy, P_ref;
    T dr_cs2;                         // cs2 (rho_a - rho_b)/(phi_a - phi_b)
};

// Per-simulation constants (device memory; read once per workgroup).
struct SimDev {
    int32_t nx, ny;
    int32_t tile0, ntiles;  // first tile and tile count of this sim
    int64_t off;            // element offset of the sim's population block
    int64_t ushape_off;     // element offset of the prescribed-velocity shapes
    uint32_t node_base;     // first global node index (random streams)
    int32_t uniform_rho, uniform_nu;
    int32_t row0;           // rows of all earlier simulations (inventory partials)
    double W, phi_a, phi_b, inv_dphi, phim;
    double theta_k, thetac_k;  // 4/W and 8/W
    double M_phi, D_s, omega_k, omega_c;
    double rho_b, drho, nu_b, dnu, omega_zeta;
    double sigma0, beta, c_max, ks;
    double u_wall, F_ext_x, F_ext_y, vel_period_T;
    double P_ref;
    double qref_f;                     // phi reference of the f storage (0 unless FP16)
    double scale_f, scale_h, scale_g;  // storage scales (powers of two)
    PhysConsts<double> kd;
    PhysConsts<float> kf;
};

template <class T>
struct K {
    static constexpr T cs2 = T(1) / T(3);
    static constexpr T cs4 = T(1) / T(9);
    static constexpr T third = T(1) / T(3);
    static constexpr T twelfth = T(1) / T(12);
};

// rest weights
template <class T>
__device__ __forceinline__ constexpr T wgt(int a) {
    return a == 0 ? T(4) / T(9) : (a < 5 ? T(1) / T(9) : T(1) / T(36));
}
// 1/w_a, exact in binary: 9/4, 9, 36
template <class T>
__device__ __forceinline__ constexpr T inv_wgt(int a) {
    return a == 0 ? T(2.25) : (a < 5 ? T(9) : T(36));
}
__device__ __forceinline__ constexpr int EXa(int a) {
    return (a == 1 || a == 5 || a == 8) ? 1 : ((a == 3 || a == 6 || a == 7) ? -1 : 0);
}
__device__ __forceinline__ constexpr int EYa(int a) {
    return (a == 2 || a == 5 || a == 6) ? 1 : ((a == 4 || a == 7 || a == 8) ? -1 : 0);
}
__device__ __forceinline__ constexpr int OPPa(int a) {
    return a == 0 ? 0 : (a < 5 ? ((a + 1) % 4) + 1 : ((a - 5 + 2) % 4) + 5);
}

// ---------------------------------------------------------------------------
// Raw moments (App. A, matrix P) of nine values.
// ---------------------------------------------------------------------------
template <class T>
struct Raw6 {
    T m0, m1, m2, m3, m4, m5;
};

template <class T>
__device__ __forceinline__ Raw6<T> raw_moments6(const T d[9]) {
    const T a13 = d[1] + d[3], s13 = d[1] - d[3];
    const T a24 = d[2] + d[4], s24 = d[2] - d[4];
    const T a56 = d[5] + d[6], s56 = d[5] - d[6];
    const T a78 = d[7] + d[8], s78 = d[7] - d[8];
    const T d4 = a56 + a78;
    Raw6<T> m;
    m.m0 = ((d[0] + a13) + a24) + d4;
    m.m1 = s13 + s56 - s78;       // d1 - d3 + d5 - d6 - d7 + d8
    m.m2 = s24 + a56 - a78;       // d2 - d4 + d5 + d6 - d7 - d8
    m.m3 = a13 + d4;
    m.m4 = a24 + d4;
    m.m5 = s56 + s78;             // d5 - d6 + d7 - d8
    return m;
}

// Zeroth moment with the same association as m0 in raw_moments3/6, so a
// node's phi, c and P^ carry the same bits whether computed as a tile
// interior node or as a halo node of a neighbouring tile.
template <class T>
__device__ __forceinline__ T sum9(const T d[9]) {
    return ((d[0] + (d[1] + d[3])) + (d[2] + d[4])) + ((d[5] + d[6]) + (d[7] + d[8]));
}

template <class T>
__device__ __forceinline__ void raw_moments3(const T d[9], T& m0, T& m1, T& m2) {
    const T a13 = d[1] + d[3], s13 = d[1] - d[3];
    const T a24 = d[2] + d[4], s24 = d[2] - d[4];
    const T a56 = d[5] + d[6], s56 = d[5] - d[6];
    const T a78 = d[7] + d[8], s78 = d[7] - d[8];
    m0 = ((d[0] + a13) + a24) + (a56 + a78);
    m1 = s13 + s56 - s78;
    m2 = s24 + a56 - a78;
}

// Moments of a scalar lattice from its stored values v_a (= q_a/w_a up to
// the storage offset and scale): zeroth moment sum_a w_a v_a written as
// v_0 + sum_a w_a (v_a - v_0), and the first moments sum_a w_a e_a v_a with
// pairwise differences.  Both are exact when all v_a are equal, so a node at
// rest in a bulk phase reproduces its own bits every step (no drift of the
// bulk values through rounding).
// EXACT (FP32 storage): the weights enter as one correctly rounded division
// by 36 of an integer-weighted sum rather than as products with the rounded
// 1/9 and 1/36, whose common bias would scale the moments by 1 + 7.45e-9.
template <class T, bool EXACT = false>
__device__ __forceinline__ void scalar_moments(const T v[9], T& m0, T& m1, T& m2) {
    const T v4 = T(4) * v[0];
    const T A = (v[1] + v[2]) + (v[3] + v[4]);
    const T B = (v[5] + v[6]) + (v[7] + v[8]);
    if constexpr (EXACT) {
        m0 = v[0] + div_const<36>(T(4) * (A - v4) + (B - v4));
        m1 = div_const<36>(T(4) * (v[1] - v[3]) + ((v[5] - v[6]) + (v[8] - v[7])));
        m2 = div_const<36>(T(4) * (v[2] - v[4]) + ((v[5] + v[6]) - (v[7] + v[8])));
    } else {
        m0 = v[0] + (T(4) * (A - v4) + (B - v4)) * T(1.0 / 36.0);
        m1 = (v[1] - v[3]) * T(1.0 / 9.0) + ((v[5] - v[6]) + (v[8] - v[7])) * T(1.0 / 36.0);
        m2 = (v[2] - v[4]) * T(1.0 / 9.0) + ((v[5] + v[6]) - (v[7] + v[8])) * T(1.0 / 36.0);
    }
}

// P^-1 applied to a raw-moment deviation dr, scaled by scale/w_a: the change
// of the stored values relative to the rest equilibrium of the node's own
// zeroth moment.
template <class T>
__device__ __forceinline__ void pinv_dev(const T r[9], T scale, T s[9]) {
    const T c0 = scale * T(2.25);
    const T c1 = scale * T(4.5);
    const T c5 = scale * T(9);
    const T r37 = r[3] - r[8], r48 = r[4] - r[8];
    s[0] = (r[0] - r[3] - r[4] + r[8]) * c0;
    s[1] = (r[1] + r37 - r[7]) * c1;
    s[2] = (r[2] + r48 - r[6]) * c1;
    s[3] = (-r[1] + r37 + r[7]) * c1;
    s[4] = (-r[2] + r48 + r[6]) * c1;
    const T p56 = r[5] + r[8], m56 = r[8] - r[5];
    s[5] = (p56 + r[6] + r[7]) * c5;
    s[6] = (m56 + r[6] - r[7]) * c5;
    s[7] = (p56 - r[6] - r[7]) * c5;
    s[8] = (m56 - r[6] + r[7]) * c5;
}
// The same map for FP32 values evaluated in FP64 (the same expressions, so
// the same bits as pinv_dev<double> of the widened values), each result
// rounded to FP32 once.
__device__ __forceinline__ void pinv_dev_wide(const float r[9], float scale, float s[9]) {
    const double c0 = double(scale) * 2.25;
    const double c1 = double(scale) * 4.5;
    const double c5 = double(scale) * 9.0;
    const double r1 = r[1], r2 = r[2], r3 = r[3], r4 = r[4], r5 = r[5], r6 = r[6], r7 = r[7],
                 r8 = r[8];
    const double r37 = r3 - r8, r48 = r4 - r8;
    s[0] = float((double(r[0]) - r3 - r4 + r8) * c0);
    s[1] = float((r1 + r37 - r7) * c1);
    s[2] = float((r2 + r48 - r6) * c1);
    s[3] = float((-r1 + r37 + r7) * c1);
    s[4] = float((-r2 + r48 + r6) * c1);
    const double p56 = r5 + r8, m56 = r8 - r5;
    s[5] = float((p56 + r6 + r7) * c5);
    s[6] = float((m56 + r6 - r7) * c5);
    s[7] = float((p56 - r6 - r7) * c5);
    s[8] = float((m56 - r6 + r7) * c5);
}
// the same added to base (the node's zeroth moment in storage units), in
// one expression per value so that each is a single multiply-add
template <class T>
__device__ __forceinline__ void pinv_dev_add(const T r[9], T scale, T base, T s[9]) {
    const T c0 = scale * T(2.25);
    const T c1 = scale * T(4.5);
    const T c5 = scale * T(9);
    const T r37 = r[3] - r[8], r48 = r[4] - r[8];
    s[0] = base + (r[0] - r[3] - r[4] + r[8]) * c0;
    s[1] = base + (r[1] + r37 - r[7]) * c1;
    s[2] = base + (r[2] + r48 - r[6]) * c1;
    s[3] = base + (-r[1] + r37 + r[7]) * c1;
    s[4] = base + (-r[2] + r48 + r[6]) * c1;
    const T p56 = r[5] + r[8], m56 = r[8] - r[5];
    s[5] = base + (p56 + r[6] + r[7]) * c5;
    s[6] = base + (m56 + r[6] - r[7]) * c5;
    s[7] = base + (p56 - r[6] - r[7]) * c5;
    s[8] = base + (m56 - r[6] + r[7]) * c5;
}

// Scalar lattices f, h: deviation of the post-collision raw moments
// F^-1(u) kappa~ from the rest moments s (1, 0, 0, cs2, cs2, 0, 0, 0, cs2^2),
// kappa~ = (s, k1, k2, cs2 s, cs2 s, 0, 0, 0, cs2^2 s).  Without flow only
// the first-order entries remain.
template <class T, bool MOVING>
__device__ __forceinline__ void scalar_post_dev(T s, T k1, T k2, T ux, T uy, T r[9]) {
    if (!MOVING) {
        r[0] = T(0); r[1] = k1; r[2] = k2; r[3] = T(0); r[4] = T(0);
        r[5] = T(0); r[6] = T(0); r[7] = T(0); r[8] = T(0);
        return;
    }
    const T a = K<T>::cs2 * s;
    r[0] = T(0);
    r[1] = ux * s + k1;
    r[2] = uy * s + k2;
    r[3] = ux * (ux * s + T(2) * k1);
    r[4] = uy * (uy * s + T(2) * k2);
    const T r5 = ux * uy * s + uy * k1 + ux * k2;
    r[5] = r5;
    r[6] = ux * (r5 + uy * k1) + uy * a;
    r[7] = uy * (r5 + ux * k2) + ux * a;
    r[8] = ux * uy * (r5 + uy * k1 + ux * k2) + (ux * ux + uy * uy) * a;
}

// ---------------------------------------------------------------------------
// P^-1 (App. A) fused with the storage encoding s_a = q_a (scale/w_a) - bias.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void pinv_encode(const T r[9], T scale, T bias, T s[9]) {
    const T c0 = scale * T(2.25);
    const T c1 = scale * T(4.5);  // (1/2) * 9
    const T c5 = scale * T(9);    // (1/4) * 36
    const T r37 = r[3] - r[8], r48 = r[4] - r[8];
    s[0] = (r[0] - r[3] - r[4] + r[8]) * c0 - bias;
    s[1] = (r[1] + r37 - r[7]) * c1 - bias;
    s[2] = (r[2] + r48 - r[6]) * c1 - bias;
    s[3] = (-r[1] + r37 + r[7]) * c1 - bias;
    s[4] = (-r[2] + r48 + r[6]) * c1 - bias;
    const T p56 = r[5] + r[8], m56 = r[8] - r[5];
    s[5] = (p56 + r[6] + r[7]) * c5 - bias;
    s[6] = (m56 + r[6] - r[7]) * c5 - bias;
    s[7] = (p56 - r[6] - r[7]) * c5 - bias;
    s[8] = (m56 - r[6] + r[7]) * c5 - bias;
}

// ---------------------------------------------------------------------------
// Scalar lattices f, h: post-collision raw moments r = F^-1(u) kappa~ with
// kappa~ = (s, k1, k2, cs2 s, cs2 s, 0, 0, 0, cs2^2 s) (App. C / Sec. 3).
// ---------------------------------------------------------------------------
template <class T, bool MOVING>
__device__ __forceinline__ void scalar_post_raw(T s, T k1, T k2, T ux, T uy, T r[9]) {
    const T a = K<T>::cs2 * s;
    if (!MOVING) {
        r[0] = s; r[1] = k1; r[2] = k2; r[3] = a; r[4] = a;
        r[5] = T(0); r[6] = T(0); r[7] = T(0); r[8] = K<T>::cs2 * a;
        return;
    }
    r[0] = s;
    r[1] = ux * s + k1;
    r[2] = uy * s + k2;
    r[3] = ux * (ux * s + T(2) * k1) + a;
    r[4] = uy * (uy * s + T(2) * k2) + a;
    const T r5 = ux * uy * s + uy * k1 + ux * k2;
    r[5] = r5;
    r[6] = ux * (r5 + uy * k1) + uy * a;
    r[7] = uy * (r5 + ux * k2) + ux * a;
    r[8] = ux * uy * (r5 + uy * k1 + ux * k2) + (ux * ux + uy * uy + K<T>::cs2) * a;
}

// ---------------------------------------------------------------------------
// Flow lattice g: post-collision central moments in deviation form
// (t = eta~ - rest, rest = P_ref (1,0,0,cs2,cs2,0,0,0,cs2^2)) mapped to
// deviation raw moments with F^-1(u) (App. B).
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void flow_post_raw(const T t[9], T ux, T uy, T Pref, T r[9]) {
    const T T00 = t[0] + Pref;
    const T T20 = t[3] + K<T>::cs2 * Pref;
    const T T02 = t[4] + K<T>::cs2 * Pref;
    const T uxuy = ux * uy, ux2 = ux * ux, uy2 = uy * uy;
    r[0] = t[0];
    r[1] = ux * T00 + t[1];
    r[2] = uy * T00 + t[2];
    r[3] = ux2 * T00 + T(2) * ux * t[1] + t[3];
    r[4] = uy2 * T00 + T(2) * uy * t[2] + t[4];
    r[5] = uxuy * T00 + uy * t[1] + ux * t[2] + t[5];
    r[6] = ux2 * uy * T00 + T(2) * uxuy * t[1] + ux2 * t[2] + uy * T20 + T(2) * ux * t[5] + t[6];
    r[7] = ux * uy2 * T00 + uy2 * t[1] + T(2) * uxuy * t[2] + ux * T02 + T(2) * uy * t[5] + t[7];
    r[8] = ux2 * uy2 * T00 + T(2) * ux * uy2 * t[1] + T(2) * ux2 * uy * t[2] + uy2 * T20 +
           ux2 * T02 + T(4) * uxuy * t[5] + T(2) * uy * t[6] + T(2) * ux * t[7] + t[8];
}

// Equilibrium central moments of g in deviation form (App. D, first-order
// entries with the sign -psi u).
template <class T>
__device__ __forceinline__ void flow_eq_dev(T dP, T psi, T ux, T uy, T t[9]) {
    const T ux2 = ux * ux, uy2 = uy * uy;
    const T cs2 = K<T>::cs2;
    t[0] = dP;
    t[1] = -psi * ux;
    t[2] = -psi * uy;
    t[3] = cs2 * dP + psi * ux2;
    t[4] = cs2 * dP + psi * uy2;
    t[5] = psi * ux * uy;
    t[6] = -psi * (ux2 + cs2) * uy;
    t[7] = -psi * (uy2 + cs2) * ux;
    t[8] = K<T>::cs4 * dP + psi * (cs2 * (ux2 + uy2) + ux2 * uy2);
}

// Collision of g (App. D).  m: raw deviation moments of the pre-collision
// populations; P_hat = P_ref + m0.  (fpx, fpy) = -grad psi^, (ftx, fty) the
// total force.  Returns the post-collision deviation central moments t.
template <class T>
__device__ __forceinline__ void flow_collide(const Raw6<T>& m, T ux, T uy, T dP, T psi, T P_hat,
                                             T fpx, T fpy, T ftx, T fty, T gam, T omega_zeta,
                                             T omega_nu, T t[9]) {
    const T cs2 = K<T>::cs2;
    const T ux2 = ux * ux, uy2 = uy * uy, uxuy = ux * uy;
    // pre-collision second-order central moments minus their rest values
    const T a20 = m.m3 - T(2) * ux * m.m1 + ux2 * P_hat;
    const T a02 = m.m4 - T(2) * uy * m.m2 + uy2 * P_hat;
    const T a11 = m.m5 - ux * m.m2 - uy * m.m1 + uxuy * P_hat;
    // sources (App. D)
    const T s10 = cs2 * ftx - ux * gam;
    const T s01 = cs2 * fty - uy * gam;
    const T s20 = T(2) * cs2 * fpx * ux + (ux2 + cs2) * gam;
    const T s02 = T(2) * cs2 * fpy * uy + (uy2 + cs2) * gam;
    const T s11 = cs2 * (fpx * uy + fpy * ux) + uxuy * gam;
    // bulk/shear split B
    const T e2s = a20 + a02, e2d = a20 - a02;
    const T q2s = T(2) * cs2 * dP + psi * (ux2 + uy2);
    const T q2d = psi * (ux2 - uy2);
    const T q11 = psi * uxuy;
    const T t2s = e2s + omega_zeta * (q2s - e2s) + (T(1) - T(0.5) * omega_zeta) * (s20 + s02);
    const T t2d = e2d + omega_nu * (q2d - e2d) + (T(1) - T(0.5) * omega_nu) * (s20 - s02);
    const T t11 = a11 + omega_nu * (q11 - a11) + (T(1) - T(0.5) * omega_nu) * s11;
    t[0] = dP + T(0.5) * gam;
    t[1] = -psi * ux + T(0.5) * s10;
    t[2] = -psi * uy + T(0.5) * s01;
    t[3] = T(0.5) * (t2s + t2d);
    t[4] = T(0.5) * (t2s - t2d);
    t[5] = t11;
    t[6] = -psi * (ux2 + cs2) * uy;
    t[7] = -psi * (uy2 + cs2) * ux;
    t[8] = K<T>::cs4 * dP + psi * (cs2 * (ux2 + uy2) + ux2 * uy2);
}

// Isotropic nine-point gradient on an LDS tile with row pitch P:
// d_i Phi = (1/cs2) sum_a w_a e_ai Phi(x + e_a).
template <class T, int P>
__device__ __forceinline__ void lds_grad(const T* L, int idx, T& gx, T& gy) {
    const T e = L[idx + 1], w = L[idx - 1];
    const T n = L[idx + P], s = L[idx - P];
    const T ne = L[idx + P + 1], nw = L[idx + P - 1];
    const T se = L[idx - P + 1], sw = L[idx - P - 1];
    gx = (e - w) * K<T>::third + ((ne - nw) + (se - sw)) * K<T>::twelfth;
    gy = (n - s) * K<T>::third + ((ne + nw) - (se + sw)) * K<T>::twelfth;
}

}  // namespace cmlb
