// HIP kernels of the three-dimensional (D3Q27) coupled central-moment LB
// step for gfx950.  The paper states its schemes in 2D and only claims the
// extension; the 3D scheme here takes each 2D step over axis by axis
// (D3Q27 = D1Q3 x D1Q3 x D1Q3), with the readings listed in the design notes.
//
// A time step is two launches over a tile table of every simulation:
//
//   k_moments3  pull the 81 pre-collision populations of each node,
//               q_a(x) = q~_a(x - e_a) (own opposite slot behind a wall),
//               and keep only what the collision needs: zeroth and first
//               moments of f and h, moments up to second order of g
//               (18 values per node, in the compute type);
//   k_collide3  per column of 64 x TY nodes marching along z: phi (radius
//               2), c and P^ (radius 1) planes from the moment arrays into
//               LDS rings, unit normals on the radius-1 plane, then per node
//               the interface geometry, Langmuir sigma(c), F_s, F_p, u, P
//               and the three collisions; post-collision populations stored
//               at the node (aligned).
//
// Splitting at the moments replaces the fused 2D kernel's halo ring, which
// in 3D would pull 27 populations for 2-5 halo nodes per own node, by
// coalesced reads of three compact fields; it costs 2 x 72 bytes per node
// (FP32) on top of the 648 algorithmic bytes.
//
// Storage is the 2D library's: s_a = (q_a/w_a - q_ref) scale per population,
// q_ref = phi_m (FP16 f), P_ref = rho_b cs2 (g), 0 otherwise.  Collisions
// work on deviations from the rest state, so FP32 keeps its relative
// precision on small velocities, and outputs are the node's own zeroth
// moment plus a deviation, so a resting bulk node is a fixed point.  With FP32
// storage the weights enter as 27 w_a (exact) with one correctly rounded
// division by 27 per moment, and the flow collision changes the momentum by
// exactly cs2 F, as in 2D.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "device_common.hpp"

namespace cmlb3 {

using cmlb::Buf;
using cmlb::CPOL_NT;
using cmlb::div_const;
using cmlb::fmix32;
using cmlb::log_;
using cmlb::make_rsrc;
using cmlb::mirror_coord;
using cmlb::rcp_;
using cmlb::sqrt_;
using cmlb::Store;
using cmlb::weyl;
using cmlb::wrap_coord;

constexpr int FLOW_NONE = 0, FLOW_PRESCRIBED = 1, FLOW_COUPLED = 2;
constexpr int NMOM = 18;         // moments kept per node
constexpr int TXW = 64;          // tile width (one wavefront)
constexpr int WG3 = 256;         // threads per block of the auxiliary kernels
constexpr double NORMAL_EPS3 = 1e-12;

template <class T>
struct C3 {
    static constexpr T cs2 = T(1) / T(3);
    static constexpr T w0 = T(8) / T(27);    // rest
    static constexpr T w1 = T(2) / T(27);    // faces
    static constexpr T w2 = T(1) / T(54);    // edges
    static constexpr T w3 = T(1) / T(216);   // corners
};

// Direction a = ix + 3 iy + 9 iz, i -> e: 0 -> 0, 1 -> +1, 2 -> -1.
__device__ __forceinline__ constexpr int E1(int i) { return i == 0 ? 0 : (i == 1 ? 1 : -1); }
__device__ __forceinline__ constexpr int EXd(int a) { return E1(a % 3); }
__device__ __forceinline__ constexpr int EYd(int a) { return E1((a / 3) % 3); }
__device__ __forceinline__ constexpr int EZd(int a) { return E1(a / 9); }
__device__ __forceinline__ constexpr int OPPd(int a) {
    // opposite component index: 0 -> 0, 1 <-> 2
    return ((3 - a % 3) % 3) + 3 * ((3 - (a / 3) % 3) % 3) + 9 * ((3 - a / 9) % 3);
}
template <class T>
__device__ __forceinline__ constexpr T wgt3(int a) {
    const int n = (a % 3 != 0) + ((a / 3) % 3 != 0) + (a / 9 != 0);
    return n == 0 ? C3<T>::w0 : (n == 1 ? C3<T>::w1 : (n == 2 ? C3<T>::w2 : C3<T>::w3));
}
// Per-simulation constants in the compute type.
template <class T>
struct Consts3 {
    T inv_f, qref_f, scale_f, inv_h, scale_h, inv_g, scale_g;
    T wdec3[4];  // w_a / scale_g for n = 0..3 non-zero components (scaled g)
    T phi_a, phi_b, inv_dphi, phim, theta_k, thetac_k;
    T M_phi, D_s, omega_k, omega_c;
    T rho_b, drho, nu_b, dnu, inv_rho_b, omega_nu_b, omega_zeta;
    T sigma0, beta, c_max, inv_cmax, ks, u_wall, Fx, Fy, Fz, P_ref, dr_cs2;
    // storage encoding of a post-collision population with n non-zero
    // direction components as left by inverse27: scale / w_a / 2^n (read by
    // the binary16 kernels; FP32 and FP64 storage is unscaled)
    T enc_f[4], enc_h[4], enc_g[4];
};

struct SimDev3 {
    int32_t nx, ny, nz;
    int32_t uniform_rho, uniform_nu;
    int64_t off;         // element offset of this sim's populations (3 x 27 planes)
    int64_t moff;        // element offset of its moments (18 planes)
    int64_t uoff;        // element offset of its prescribed velocity shapes (3 planes)
    uint32_t node_base;  // first global node index (stochastic-rounding seed)
    uint32_t pad2_;
    double vel_period_T;
    Consts3<double> kd;
    Consts3<float> kf;
};

template <class T>
__device__ __forceinline__ const Consts3<T>& consts3(const SimDev3* sd);
template <>
__device__ __forceinline__ const Consts3<double>& consts3<double>(const SimDev3* sd) {
    return sd->kd;
}
template <>
__device__ __forceinline__ const Consts3<float>& consts3<float>(const SimDev3* sd) {
    return sd->kf;
}

struct StepArgs3 {
    const void* src;       // populations read (pre-collision, pull form)
    void* dst;             // populations written
    void* mom;             // moments arena (compute type)
    const SimDev3* sims;
    const int4* tiles;     // (sim, x0, y0, z0)
    int32_t tile_base, ntiles;
    int32_t xcd_remap;
    int32_t zseg;          // collision: z planes per column segment
    const void* ushape;    // prescribed velocity shapes, compute type
    const int64_t* step_in;
    int64_t* step_out;
    int32_t* fault;
    double* fields_out;    // fields mode: [6][nz][ny][nx] (phi, c, ux, uy, uz, P)
};

__device__ __forceinline__ int tile_index(const StepArgs3& a) {
    int tix = blockIdx.x;
    if (a.xcd_remap) {
        // XCD k (blocks k, k+8, ...) takes the contiguous tile range
        // [k*per, (k+1)*per), so neighbouring tiles share one L2
        const int per = (int)gridDim.x >> 3;
        tix = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    }
    return tix;
}

// ---------------------------------------------------------------------------
// k_moments3: pulled populations -> moments.
// Tile = 64 x MT_ROWS nodes (x by (y, z) rows); block = 256 threads.
// Moment planes (per node, compute type):
//   0 f zeroth (storage units), 1-3 f first (true units),
//   4 h zeroth (storage units), 5-7 h first,
//   8 g zeroth of the deviation (P^ - P_ref), 9-11 g first,
//   12-14 g second diagonal (xx, yy, zz), 15-17 g second off-diagonal
//   (xy, xz, yz), all of the deviations d_a = g_a - w_a P_ref.
// ---------------------------------------------------------------------------
constexpr int MT_ROWS = 4;  // (y, z) rows per moments tile

// stored values of the 27 pulled populations, as register words
template <class S, bool WALLS>
__device__ __forceinline__ void pull27(__amdgpu_buffer_rsrc_t r, int pb, int x, int y, int z,
                                       int nx, int ny, int nz, bool inner,
                                       typename Buf<S>::word v[27]) {
    constexpr int SB = sizeof(S);
    const int plane = nx * ny;
    if (inner) {
        // rows y - 1 .. y + 1 and planes z - 1 .. z + 1 in the grid; the
        // periodic wrap in x per lane: column 0 pulls e_x = +1 from column
        // nx - 1, column nx - 1 pulls e_x = -1 from column 0
        const int vo = ((z * ny + y) * nx + x) * SB;
        const int xp = x == 0 ? vo + nx * SB : vo;
        const int xm = x == nx - 1 ? vo - nx * SB : vo;
#pragma unroll
        for (int a = 0; a < 27; ++a) {
            const int so = a * pb - (EXd(a) + EYd(a) * nx + EZd(a) * plane) * SB;
            v[a] = Buf<S>::raw(r, EXd(a) > 0 ? xp : (EXd(a) < 0 ? xm : vo), so);
        }
        return;
    }
#pragma unroll
    for (int a = 0; a < 27; ++a) {
        int sx = x - EXd(a), sy = y - EYd(a), sz = z - EZd(a), pa = a;
        sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
        sz = sz < 0 ? sz + nz : (sz >= nz ? sz - nz : sz);
        if (sy < 0 || sy >= ny) {
            if (WALLS) {
                pa = OPPd(a);
                sx = x;
                sy = y;
                sz = z;
            } else {
                sy = sy < 0 ? sy + ny : sy - ny;
            }
        }
        // the plane varies per lane at a wall, so it goes into the vector offset
        v[a] = Buf<S>::raw(r, ((sz * ny + sy) * nx + sx) * SB + pa * pb, 0);
    }
}

// zeroth (exact for a uniform node: s0 + sum w (s_a - s0)) and first
// moments of stored scalar-lattice values, storage units
// 27 w_a: 8, 2, 1/2, 1/8 for 0, 1, 2, 3 non-zero components (exact)
template <class T>
__device__ __forceinline__ constexpr T wgt3x27(int a) {
    return T(8) / T(1 << (2 * ((a % 3 != 0) + ((a / 3) % 3 != 0) + (a / 9 != 0))));
}
// EXACT (FP32 storage): the weights enter as 27 w_a (exact) and one
// correctly rounded division by 27 per moment, not as products with the
// rounded weights, whose common bias would scale the moments every step
template <class T, bool EXACT = false>
__device__ __forceinline__ void scalar_moments27(const T v[27], T& m0, T& jx, T& jy, T& jz) {
#pragma clang fp contract(off)
    const T s0 = v[0];
    T z = T(0), x = T(0), y = T(0), w = T(0);
#pragma unroll
    for (int a = 1; a < 27; ++a) {
        const T d = EXACT ? wgt3x27<T>(a) * (v[a] - s0) : wgt3<T>(a) * (v[a] - s0);
        z += d;
        if (EXd(a)) x += EXd(a) > 0 ? d : -d;
        if (EYd(a)) y += EYd(a) > 0 ? d : -d;
        if (EZd(a)) w += EZd(a) > 0 ? d : -d;
    }
    if constexpr (EXACT) {
        z = div_const<27>(z);
        x = div_const<27>(x);
        y = div_const<27>(y);
        w = div_const<27>(w);
    }
    m0 = s0 + z;
    jx = x;
    jy = y;
    jz = w;
}

template <class S, class T, int FLOW, bool WALLS>
__global__ __launch_bounds__(WG3) void k_moments3(const StepArgs3 a) {
    const int tix = tile_index(a);
    if (tix >= a.ntiles) return;
    const int4 tl = a.tiles[a.tile_base + tix];
    const SimDev3* sd = a.sims + tl.x;
    // constants by value: read once, before any store (a store could alias
    // the table for all the compiler knows)
    const Consts3<T> k = consts3<T>(sd);
    const int nx = sd->nx, ny = sd->ny, nz = sd->nz;
    // a moments tile is 64 columns of MT_ROWS consecutive (y, z) rows,
    // rows numbered z ny + y; tl.z is its first row
    const int x = tl.y + (int)(threadIdx.x & 63);
    const int rr = tl.z + (int)(threadIdx.x >> 6);
    if (x >= nx || rr >= ny * nz) return;
    const int y = rr % ny, z = rr / ny;
    constexpr int SB = sizeof(S);
    constexpr bool CPL = FLOW == FLOW_COUPLED;
    const int plane = nx * ny;
    const int vol = plane * nz;
    const int pb = vol * SB;
    const int lb = 27 * pb;
    const char* srcb = static_cast<const char*>(a.src) + sd->off * SB;
    // a wave holds one (y, z) row: the general path only for the rows next
    // to the y and z ends of the grid
    const bool inner = y >= 1 && y + 1 < ny && z >= 1 && z + 1 < nz;
    T* mom = static_cast<T*>(a.mom) + sd->moff + ((z * ny + y) * nx + x);
    // all pulls before the first store: a load issued after a store would
    // wait for that store as well.  Binary16 values are widened only after
    // all three lattices' pulls have been issued: widening inside a pull's
    // branch made a wave wait for one lattice's 27 loads before it issued
    // the next 27 (with the 81 in flight the 256x128x128 drop steps 4.7%
    // faster).  FP32 and FP64 need no widening, and the compiler already
    // issues their 81 pulls ahead of the moment sums.
    constexpr bool AHEAD = Store<S>::scaled;
    using W = typename Buf<S>::word;
    W sf[27], sh[AHEAD ? 27 : 1], sg[AHEAD && CPL ? 27 : 1];
    T v[27], fm[4], hm[4];
    pull27<S, WALLS>(make_rsrc(srcb, lb), pb, x, y, z, nx, ny, nz, inner, sf);
    if constexpr (AHEAD) {
        pull27<S, WALLS>(make_rsrc(srcb + lb, lb), pb, x, y, z, nx, ny, nz, inner, sh);
        if constexpr (CPL)
            pull27<S, WALLS>(make_rsrc(srcb + 2 * (int64_t)lb, lb), pb, x, y, z, nx, ny, nz, inner, sg);
    }
#pragma unroll
    for (int q = 0; q < 27; ++q) v[q] = T(Buf<S>::widen(sf[q]));
    scalar_moments27<T, std::is_same_v<S, float>>(v, fm[0], fm[1], fm[2], fm[3]);
    if constexpr (AHEAD) {
#pragma unroll
        for (int q = 0; q < 27; ++q) v[q] = T(Buf<S>::widen(sh[q]));
    } else {
        pull27<S, WALLS>(make_rsrc(srcb + lb, lb), pb, x, y, z, nx, ny, nz, inner, v);
    }
    scalar_moments27<T, std::is_same_v<S, float>>(v, hm[0], hm[1], hm[2], hm[3]);
    T r0 = T(0), r1[3] = {T(0), T(0), T(0)}, r2[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    if constexpr (CPL) {
        if constexpr (AHEAD) {
#pragma unroll
            for (int q = 0; q < 27; ++q) v[q] = T(Buf<S>::widen(sg[q]));
        } else {
            pull27<S, WALLS>(make_rsrc(srcb + 2 * (int64_t)lb, lb), pb, x, y, z, nx, ny, nz, inner, v);
        }
        // deviations d_a = w_a s_a / scale and their raw moments
        {
#pragma clang fp contract(off)
#pragma unroll
        for (int q = 0; q < 27; ++q) {
            // binary16: one product with w_a / scale_g (scale_g a power of
            // two, so the same bits as w_a (v / scale_g))
            const T d = std::is_same_v<S, float> ? wgt3x27<T>(q) * v[q]
                        : (Store<S>::scaled ? v[q] * k.wdec3[(q % 3 != 0) + ((q / 3) % 3 != 0) + (q / 9 != 0)]
                                            : wgt3<T>(q) * v[q]);
            const int ex = EXd(q), ey = EYd(q), ez = EZd(q);
            r0 += d;
            if (ex) r1[0] += ex > 0 ? d : -d;
            if (ey) r1[1] += ey > 0 ? d : -d;
            if (ez) r1[2] += ez > 0 ? d : -d;
            if (ex) r2[0] += d;
            if (ey) r2[1] += d;
            if (ez) r2[2] += d;
            if (ex && ey) r2[3] += ex * ey > 0 ? d : -d;
            if (ex && ez) r2[4] += ex * ez > 0 ? d : -d;
            if (ey && ez) r2[5] += ey * ez > 0 ? d : -d;
        }
        if constexpr (std::is_same_v<S, float>) {
            r0 = div_const<27>(r0);
#pragma unroll
            for (int i = 0; i < 3; ++i) r1[i] = div_const<27>(r1[i]);
#pragma unroll
            for (int i = 0; i < 6; ++i) r2[i] = div_const<27>(r2[i]);
        }
        }
    }
    mom[0] = fm[0];
    mom[vol] = fm[1] * k.inv_f;
    mom[2 * vol] = fm[2] * k.inv_f;
    mom[3 * vol] = fm[3] * k.inv_f;
    mom[4 * vol] = hm[0];
    mom[5 * vol] = hm[1] * k.inv_h;
    mom[6 * vol] = hm[2] * k.inv_h;
    mom[7 * vol] = hm[3] * k.inv_h;
    if constexpr (CPL) {
        mom[8 * vol] = r0;
#pragma unroll
        for (int i = 0; i < 3; ++i) mom[(9 + i) * vol] = r1[i];
#pragma unroll
        for (int i = 0; i < 6; ++i) mom[(12 + i) * vol] = r2[i];
    }
}

// ---------------------------------------------------------------------------
// Axis-wise inverse of the central-moment map.  t[i + 3j + 9k] holds central
// moments with exponents (i, j, k) on entry and, on exit, the populations
// with components (E1(i), E1(j), E1(k)) times 2^n, n the number of non-zero
// components.  One axis: central -> raw (r0 = k0, r1 = k1 + u k0,
// r2 = k2 + 2u k1 + u^2 k0), raw -> populations (q0 = r0 - r2,
// 2 q+ = r2 + r1, 2 q- = r2 - r1).  The halvings are left to the storage
// encoding, which multiplies each population by a constant anyway
// (enc_wgt3); scaling by powers of two is exact, so this changes no bits.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void axis_inv(T& a0, T& a1, T& a2, T u, T u2) {
    const T r1 = a1 + u * a0;
    const T r2 = a2 + T(2) * u * a1 + u2 * a0;
    a0 = a0 - r2;
    a1 = r2 + r1;
    a2 = r2 - r1;
}
// number of non-zero components of direction a
__device__ __forceinline__ constexpr int nnz3(int a) {
    return (a % 3 != 0) + ((a / 3) % 3 != 0) + (a / 9 != 0);
}
// 1/w_a / 2^n for a direction with n non-zero components: (27/8) 2^n
template <class T>
__device__ __forceinline__ constexpr T enc_wgt3(int n) {
    return T(27) / T(8) * T(1 << n);
}
template <class T>
__device__ __forceinline__ void inverse27(T t[27], T ux, T uy, T uz) {
    const T ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
#pragma unroll
    for (int b = 0; b < 27; b += 3) axis_inv(t[b], t[b + 1], t[b + 2], ux, ux2);
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int b = i + 9 * k;
            axis_inv(t[b], t[b + 3], t[b + 6], uy, uy2);
        }
#pragma unroll
    for (int b = 0; b < 9; ++b) axis_inv(t[b], t[b + 9], t[b + 18], uz, uz2);
}

// rest-state central moments: c(0) = 1, c(1) = 0, c(2) = cs2; central
// moments of a rest distribution about u: m(0) = 1, m(1) = -u, m(2) = cs2 + u^2
template <class T>
__device__ __forceinline__ T crest3(int a) {
    return a == 0 ? T(1) : (a == 1 ? T(0) : C3<T>::cs2);
}

// prod_i m(e_i, u_i) - prod_i c(e_i) for the factors m = (1, -u, cs2 + u^2)
// and c = (1, 0, cs2): the equilibrium's departure from the rest moments,
// built axis by axis without a difference of nearly equal terms.  With D and
// C the departure and the rest product over the axes so far, one more axis
// with departure d = m - c = (0, -u, u^2) gives D' = D m + C d and C' = C c.
// FP32 arithmetic needs this form: the plain difference cs2 - (cs2 + u^2)
// keeps u^2 only to the 3e-8 absolute rounding of cs2 + u^2, the same at a
// quasi-steady node every step, and through the second- and fourth-order
// moments of g that bias reaches the velocity (1.3e-5 after 1000 steps on a
// 64x32x32 sheared drop, against 1.5e-7 with this form).
template <class T>
__device__ __forceinline__ T mdep3(int a, int b, int c, T ux, T uy, T uz) {
    const int e[3] = {a, b, c};
    const T u[3] = {ux, uy, uz};
    T D = T(0), C = T(1);
    bool zero_d = true, zero_c = false;  // D == 0, C == 0 exactly
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (e[i] == 1) {
            // m = -u, c = 0: D' = -u (D + C), C' = 0
            const T dc = zero_c ? D : (zero_d ? C : D + C);
            D = -u[i] * dc;
            zero_d = false;
            zero_c = true;
        } else if (e[i] == 2) {
            // m = cs2 + u^2, c = cs2, d = u^2
            const T u2 = u[i] * u[i];
            const T cd = zero_c ? T(0) : C * u2;
            D = zero_d ? cd : (zero_c ? D * (C3<T>::cs2 + u2) : D * (C3<T>::cs2 + u2) + cd);
            zero_d = zero_d && zero_c;
            if (!zero_c) C = C * C3<T>::cs2;
        }
    }
    return D;
}

// Scalar lattice (f or h): deviation of the post-collision central moments
// from those of the rest distribution s w_a about u, then populations:
// out_a = q~_a - w_a s.
template <class T, bool MOV>
__device__ __forceinline__ void scalar_dev27(T s, T k1x, T k1y, T k1z, T ux, T uy, T uz,
                                             T t[27]) {
    const T mx[3] = {T(1), -ux, C3<T>::cs2 + ux * ux};
    const T my[3] = {T(1), -uy, C3<T>::cs2 + uy * uy};
    const T mz[3] = {T(1), -uz, C3<T>::cs2 + uz * uz};
#pragma unroll
    for (int m = 0; m < 27; ++m) {
        const int a = m % 3, b = (m / 3) % 3, c = m / 9;
        const int order = a + b + c;
        if (order == 0) {
            t[m] = T(0);
        } else if (order == 1) {
            const T k1 = a ? k1x : (b ? k1y : k1z);
            const T u = a ? ux : (b ? uy : uz);
            t[m] = k1 + s * u;
        } else if (!MOV) {
            t[m] = T(0);  // u = 0: rest moments are the equilibrium ones
        } else {
            if constexpr (std::is_same_v<T, float>) {
                t[m] = -s * mdep3<T>(a, b, c, ux, uy, uz);
            } else {
                t[m] = s * (crest3<T>(a) * crest3<T>(b) * crest3<T>(c) - mx[a] * my[b] * mz[c]);
            }
        }
    }
    inverse27(t, ux, uy, uz);
}

// Flow lattice: post-collision central moments minus P_ref times those of
// the rest distribution, i.e. of the deviations d~_a = g~_a - w_a P_ref.
// eta2[6]: second-order central moments of the deviations (xx, yy, zz, xy,
// xz, yz); dP = P - P_ref; fp = F_p, ft = F_t, gam = F_p . u.
template <class T>
__device__ __forceinline__ void flow_dev27(const T eta2[6], T dP, T rho, T ux, T uy, T uz,
                                           const T fp[3], const T ft[3], T gam, T om_zeta,
                                           T om_nu, T t[27]) {
    const T cs2 = C3<T>::cs2;
    const T u[3] = {ux, uy, uz};
    const T mx[3] = {T(1), -ux, cs2 + ux * ux};
    const T my[3] = {T(1), -uy, cs2 + uy * uy};
    const T mz[3] = {T(1), -uz, cs2 + uz * uz};
    const T rc = rho * cs2;
    // equilibrium deviation: dP prod m + rho cs2 (prod c - prod m)
#pragma unroll
    for (int m = 0; m < 27; ++m) {
        const int a = m % 3, b = (m / 3) % 3, c = m / 9;
        const T pm = mx[a] * my[b] * mz[c];
        if constexpr (std::is_same_v<T, float>) {
            t[m] = dP * pm - rc * mdep3<T>(a, b, c, ux, uy, uz);
        } else {
            t[m] = dP * pm + rc * (crest3<T>(a) * crest3<T>(b) * crest3<T>(c) - pm);
        }
    }
    // sources (zero from third order on)
    T src[10];
    src[0] = gam;
#pragma unroll
    for (int i = 0; i < 3; ++i) src[1 + i] = cs2 * ft[i] - u[i] * gam;
#pragma unroll
    for (int i = 0; i < 3; ++i) src[4 + i] = T(2) * cs2 * fp[i] * u[i] + (u[i] * u[i] + cs2) * gam;
    src[7] = cs2 * (fp[0] * u[1] + fp[1] * u[0]) + u[0] * u[1] * gam;
    src[8] = cs2 * (fp[0] * u[2] + fp[2] * u[0]) + u[0] * u[2] * gam;
    src[9] = cs2 * (fp[1] * u[2] + fp[2] * u[1]) + u[1] * u[2] * gam;
    // rate 1 on orders 0 and 1: eq + src/2
    t[0] += T(0.5) * src[0];
    t[1] += T(0.5) * src[1];
    t[3] += T(0.5) * src[2];
    t[9] += T(0.5) * src[3];
    // second order: off-diagonal and deviatoric parts at omega_nu, trace at
    // omega_zeta
    const int od[3] = {4, 10, 12};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int m = od[i];
        t[m] = eta2[3 + i] + om_nu * (t[m] - eta2[3 + i]) + (T(1) - T(0.5) * om_nu) * src[7 + i];
    }
    const int dg[3] = {2, 6, 18};
    const T tr = eta2[0] + eta2[1] + eta2[2];
    const T tre = t[2] + t[6] + t[18];
    const T trs = src[4] + src[5] + src[6];
    const T trt = tr + om_zeta * (tre - tr) + (T(1) - T(0.5) * om_zeta) * trs;
    const T third = T(1) / T(3);
    T dd[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const T d = eta2[i] - third * tr, de = t[dg[i]] - third * tre, ds = src[4 + i] - third * trs;
        dd[i] = d + om_nu * (de - d) + (T(1) - T(0.5) * om_nu) * ds;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) t[dg[i]] = dd[i] + third * trt;
}

// Isotropic D3Q27 stencils at in-plane index idx of three LDS planes
// (z - 1, z, z + 1; row pitch PX): gradient d_i F = (1/cs2) sum_a w_a e_ai
// F(x + e_a) and divergence (1/cs2) sum_a w_a e_a . V(x + e_a).  The weights
// are products w(e_ax) w(e_ay) w(e_az) with w(0) = 2/3, w(+-1) = 1/6, so a
// component is a central difference along its axis smoothed with (1, 4, 1)
// along the other two: d_x F = (1/72) sum_jk (1,4,1)_j (1,4,1)_k
// (F(+1, j, k) - F(-1, j, k)).  The same expressions serve every node, so a
// value computed at a node carries the same bits whichever kernel instance
// (launch shape) computes it.
template <class T>
__device__ __forceinline__ T smooth3(T a, T b, T c) {
    return fma(T(4), b, a + c);
}
// F at the 26 neighbours: v[k][j][i] = F at offset (i - 1, j - 1, k - 1)
template <class T, int PX>
__device__ __forceinline__ void cube3(const T* Lm, const T* L0, const T* Lp, int idx, T v[3][3][3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T* L = k == 0 ? Lm : (k == 1 ? L0 : Lp);
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int i = 0; i < 3; ++i)
                if (i != 1 || j != 1 || k != 1) v[k][j][i] = L[idx + (i - 1) + (j - 1) * PX];
    }
}
// the three smoothed central-difference sums (72 times the gradient)
template <class T>
__device__ __forceinline__ void dsum3(const T v[3][3][3], T& sx, T& sy, T& sz) {
    T a[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        a[k] = smooth3(v[k][0][2] - v[k][0][0], v[k][1][2] - v[k][1][0], v[k][2][2] - v[k][2][0]);
    sx = smooth3(a[0], a[1], a[2]);
#pragma unroll
    for (int k = 0; k < 3; ++k)
        a[k] = smooth3(v[k][2][0] - v[k][0][0], v[k][2][1] - v[k][0][1], v[k][2][2] - v[k][0][2]);
    sy = smooth3(a[0], a[1], a[2]);
#pragma unroll
    for (int j = 0; j < 3; ++j)
        a[j] = smooth3(v[2][j][0] - v[0][j][0], v[2][j][1] - v[0][j][1], v[2][j][2] - v[0][j][2]);
    sz = smooth3(a[0], a[1], a[2]);
}
template <class T, int PX>
__device__ __forceinline__ void grad3p(const T* Lm, const T* L0, const T* Lp, int idx, T& gx,
                                       T& gy, T& gz) {
    T v[3][3][3];
    cube3<T, PX>(Lm, L0, Lp, idx, v);
    T sx, sy, sz;
    dsum3(v, sx, sy, sz);
    gx = sx * T(1.0 / 72.0);
    gy = sy * T(1.0 / 72.0);
    gz = sz * T(1.0 / 72.0);
}

// components of V are NP apart in each plane
template <class T, int PX, int NP>
__device__ __forceinline__ T div3p(const T* Vm, const T* V0, const T* Vp, int idx) {
    T v[3][3][3], sx, sy, sz, unused0, unused1;
    cube3<T, PX>(Vm, V0, Vp, idx, v);
    dsum3(v, sx, unused0, unused1);
    cube3<T, PX>(Vm + NP, V0 + NP, Vp + NP, idx, v);
    dsum3(v, unused0, sy, unused1);
    cube3<T, PX>(Vm + 2 * NP, V0 + 2 * NP, Vp + 2 * NP, idx, v);
    dsum3(v, unused0, unused1, sz);
    return ((sx + sy) + sz) * T(1.0 / 72.0);
}

// n = grad phi/(|grad phi| + eps)
template <class T>
__device__ __forceinline__ void unit3(T gx, T gy, T gz, T n[3]) {
#pragma clang fp contract(off)
    const T inv = rcp_(sqrt_(gx * gx + gy * gy + gz * gz) + T(NORMAL_EPS3));
    n[0] = gx * inv;
    n[1] = gy * inv;
    n[2] = gz * inv;
}

// A population from inverse27 in storage units, t / w_a / 2^n times the
// storage scale: binary16 takes the product from the simulation's constant
// table; FP32 and FP64 storage is unscaled, so the factor is a literal.
// encode3_add adds the result to base in the same expression (one
// multiply-add).
template <class S, class T>
__device__ __forceinline__ T encode3(T t, const T tab[4], int q) {
    if constexpr (Store<S>::scaled) return t * tab[nnz3(q)];
    else return t * enc_wgt3<T>(nnz3(q));
}
template <class S, class T>
__device__ __forceinline__ T encode3_add(T base, T t, const T tab[4], int q) {
    if constexpr (Store<S>::scaled) return base + t * tab[nnz3(q)];
    else return base + t * enc_wgt3<T>(nnz3(q));
}

// ---------------------------------------------------------------------------
// k_collide3: a column of 64 x TY nodes marching through a.zseg consecutive
// z planes, one node per thread and plane (TY waves).  Rings in LDS along z:
//   phi     4 planes of (64 + 4) x (TY + 4)   (radius 2: normals at z +- 1)
//   c, P^   4 planes of (64 + 2) x (TY + 2)   (radius 1)
//   n       3 planes x 3 components of (64 + 2) x (TY + 2)
//   grad phi of the column's own nodes, 2 planes
// Step z:  [barrier] unit normals of plane z + 1 (phi planes z .. z + 2);
//          loads of phi plane z + 3 and c, P^ plane z + 2 issued into
//          registers;  [barrier]  the node collisions of plane z, with the
//          loaded planes written into the ring slots whose planes were last
//          read before this step's first barrier.
// Memory-counter waits are in issue order (a wait for a load also waits for
// every store issued before it), so the node reads all its moments and
// hands the prefetched planes to LDS before its first population store.
// Every plane of the three fields is read from the moment arrays once per
// column, and unit normals are computed once per node of the radius-1 plane.
// ---------------------------------------------------------------------------
template <class T, int NW>
struct Occ3 {
    // waves per SIMD the register budget is sized for
    static constexpr int waves_per_eu = sizeof(T) == 4 ? (NW <= 4 ? 3 : 2) : (NW <= 4 ? 1 : 2);
};

template <class S, class T, int FLOW, bool WALLS, int TY, bool FIELDS, bool NTS>
__global__ __launch_bounds__(TY * 64, (Occ3<T, TY>::waves_per_eu)) void k_collide3(
    const StepArgs3 a) {
    constexpr int NT = TY * 64;
    constexpr int CP = NTS ? CPOL_NT : 0;
    constexpr bool CPL = FLOW == FLOW_COUPLED;
    constexpr bool MOV = FLOW != FLOW_NONE;
    constexpr int PX = TXW + 4, PY = TY + 4, PP = PX * PY;  // phi plane (radius 2)
    constexpr int QX = TXW + 2, QY = TY + 2, QP = QX * QY;  // c, P^, n plane (radius 1)
    constexpr int NPH = (PP + NT - 1) / NT;                 // phi loads per thread and plane
    constexpr int NQ = (QP + NT - 1) / NT;                  // c (P^) loads per thread and plane
    constexpr int SB = sizeof(S);
    __shared__ T phiL[4 * PP];
    __shared__ T cL[4 * QP];
    __shared__ T pL[CPL ? 4 * QP : 1];
    __shared__ T nL[CPL ? 9 * QP : 1];
    __shared__ T gL[2 * 3 * NT];

    const int tix = tile_index(a);
    if (tix >= a.ntiles) return;
    const int4 tl = a.tiles[a.tile_base + tix];
    const SimDev3* sd = a.sims + tl.x;
    // the simulation's constants by value: read once, before any store (a
    // population store could alias the table for all the compiler knows, and
    // a reload after each store would wait for that store to complete)
    const Consts3<T> k = consts3<T>(sd);
    const int nx = sd->nx, ny = sd->ny, nz = sd->nz;
    const bool uni_rho = sd->uniform_rho, uni_nu = sd->uniform_nu;
    const int64_t soff = sd->off;
    const uint32_t node_base = sd->node_base;
    const double vel_T = sd->vel_period_T;
    const int64_t uoff = sd->uoff;
    const int x0 = tl.y, y0 = tl.z, z0 = tl.w;
    const int zend = min(z0 + a.zseg, nz);
    const int plane = nx * ny, vol = plane * nz;
    const T* mom = static_cast<const T*>(a.mom) + sd->moff;
    const int64_t step = *a.step_in;
    const int tid = threadIdx.x;

    // in-plane offsets of this thread's share of the phi and c, P^ planes
    // (x periodic; y periodic or mirrored at the walls); -1 past the plane
    int po[NPH], qo[NQ];
#pragma unroll
    for (int j = 0; j < NPH; ++j) {
        const int i = tid + j * NT;
        const int ry = i / PX, rx = i - ry * PX;
        const int gx = wrap_coord(x0 - 2 + rx, nx);
        const int gy = WALLS ? mirror_coord(y0 - 2 + ry, ny) : wrap_coord(y0 - 2 + ry, ny);
        po[j] = i < PP ? gy * nx + gx : -1;
    }
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
        const int i = tid + j * NT;
        const int ry = i / QX, rx = i - ry * QX;
        const int gx = wrap_coord(x0 - 1 + rx, nx);
        const int gy = WALLS ? mirror_coord(y0 - 1 + ry, ny) : wrap_coord(y0 - 1 + ry, ny);
        qo[j] = i < QP ? gy * nx + gx : -1;
    }
    // ring slots
    auto ps = [&](int zz) { return ((zz - z0 + 2) & 3) * PP; };
    auto cs = [&](int zz) { return ((zz - z0 + 1) & 3) * QP; };
    auto ns = [&](int zz) { return ((zz - z0 + 1) % 3) * 3 * QP; };
    auto gs = [&](int zz) { return ((zz - z0) & 1) * 3 * NT; };
    auto zbase = [&](int zz) { return wrap_coord(zz, nz) * plane; };
    // plane loads are issued unconditionally at clamped addresses (in
    // bounds) and all land in registers before the first LDS write, so a
    // prologue of several planes waits for memory once
    auto load_phi = [&](int zz, T v[NPH]) {
        const int b = zbase(zz);
#pragma unroll
        for (int j = 0; j < NPH; ++j) v[j] = mom[b + max(po[j], 0)];
    };
    auto store_phi = [&](int zz, const T v[NPH]) {
        const int s = ps(zz);
#pragma unroll
        for (int j = 0; j < NPH; ++j)
            if (po[j] >= 0) phiL[s + tid + j * NT] = v[j] * k.inv_f + k.qref_f;
    };
    auto load_cp = [&](int zz, T vc[NQ], T vp[NQ]) {
        const int b = zbase(zz);
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
            vc[j] = mom[4 * vol + b + max(qo[j], 0)];
            if constexpr (CPL) vp[j] = mom[8 * vol + b + max(qo[j], 0)];
        }
    };
    auto store_cp = [&](int zz, const T vc[NQ], const T vp[NQ]) {
        const int s = cs(zz);
#pragma unroll
        for (int j = 0; j < NQ; ++j)
            if (qo[j] >= 0) {
                cL[s + tid + j * NT] = vc[j] * k.inv_h;
                if constexpr (CPL) pL[s + tid + j * NT] = vp[j];
            }
    };
    // unit normals of plane zz on the radius-1 plane (coupled) and grad phi
    // at the own nodes; needs phi planes zz - 1 .. zz + 1
    auto normals = [&](int zz) {
        const T* Lm = phiL + ps(zz - 1);
        const T* L0 = phiL + ps(zz);
        const T* Lp = phiL + ps(zz + 1);
        if constexpr (CPL) {
            T* N = nL + ns(zz);
            for (int i = tid; i < QP; i += NT) {
                const int qy = i / QX, qx = i - qy * QX;
                T g[3], n3[3];
                grad3p<T, PX>(Lm, L0, Lp, (qy + 1) * PX + qx + 1, g[0], g[1], g[2]);
                unit3(g[0], g[1], g[2], n3);
                N[i] = n3[0];
                N[QP + i] = n3[1];
                N[2 * QP + i] = n3[2];
                if (qx >= 1 && qx <= TXW && qy >= 1 && qy <= TY) {
                    const int o = (qy - 1) * TXW + qx - 1;
                    T* G = gL + gs(zz);
                    G[o] = g[0];
                    G[NT + o] = g[1];
                    G[2 * NT + o] = g[2];
                }
            }
        } else {
            const int ly = tid >> 6, lx = tid & 63;
            T g[3];
            grad3p<T, PX>(Lm, L0, Lp, (ly + 2) * PX + lx + 2, g[0], g[1], g[2]);
            T* G = gL + gs(zz);
            G[tid] = g[0];
            G[NT + tid] = g[1];
            G[2 * NT + tid] = g[2];
        }
    };

    // ---------------- prologue ---------------------------------------------
    {
        T v[4][NPH], vc[3][NQ], vp[3][NQ];
#pragma unroll
        for (int i = 0; i < 4; ++i) load_phi(z0 - 2 + i, v[i]);
#pragma unroll
        for (int i = 0; i < 3; ++i) load_cp(z0 - 1 + i, vc[i], vp[i]);
#pragma unroll
        for (int i = 0; i < 4; ++i) store_phi(z0 - 2 + i, v[i]);
#pragma unroll
        for (int i = 0; i < 3; ++i) store_cp(z0 - 1 + i, vc[i], vp[i]);
    }
    {
        T v[NPH];
        load_phi(z0 + 2, v);
        __syncthreads();
        if constexpr (CPL) normals(z0 - 1);  // only the normals of plane z0 - 1 are used
        normals(z0);
        __syncthreads();
        store_phi(z0 + 2, v);  // into the slot of plane z0 - 2
    }

    const int lx = tid & 63, ly = tid >> 6;
    const int gx = x0 + lx, gy = y0 + ly;
    const bool col_ok = gx < nx && gy < ny;
    const int pidx = (ly + 2) * PX + lx + 2;
    const int qidx = (ly + 1) * QX + lx + 1;
    if (!FIELDS && blockIdx.x == 0 && tid == 0) *a.step_out = step + 1;
    int fault = 0;

    for (int z = z0; z < zend; ++z) {
        __syncthreads();
        normals(z + 1);
        // phi plane z + 3 and c, P^ plane z + 2 into registers (issued on
        // every step, in bounds: at a segment's last step they go unused)
        T fphi[NPH], fc[NQ], fp_[NQ];
        load_phi(z + 3, fphi);
        load_cp(z + 2, fc, fp_);
        __syncthreads();
        // ... and into the ring slots of planes z - 1 (phi) and z - 2 (c, P^),
        // whose last readers passed this step's first barrier.  Called after
        // the node's LDS reads and before its population stores: waiting for
        // these loads then waits for no store of this plane.
        auto flush = [&]() {
            store_phi(z + 3, fphi);
            store_cp(z + 2, fc, fp_);
        };

        {
            // ---------------- per node ---------------------------------------
            // idle lanes of a ragged column work on clamped, in-bounds data
            // and store nothing
            const int own = z * plane + min(gy, ny - 1) * nx + min(gx, nx - 1);
            const T phi = phiL[ps(z) + pidx], c = cL[cs(z) + qidx];
            const T* G = gL + gs(z);
            const T gpx = G[tid], gpy = G[NT + tid], gpz = G[2 * NT + tid];
            const T gm2 = gpx * gpx + gpy * gpy + gpz * gpz;
            T nxv, nyv, nzv;
            if constexpr (CPL) {
                const T* N = nL + ns(z);
                nxv = N[qidx];
                nyv = N[QP + qidx];
                nzv = N[2 * QP + qidx];
            } else {
                T n3[3];
                unit3(gpx, gpy, gpz, n3);
                nxv = n3[0];
                nyv = n3[1];
                nzv = n3[2];
            }
            const T theta = k.theta_k * (k.phi_a - phi) * (phi - k.phi_b) * k.inv_dphi;
            const T theta_c = k.thetac_k * c * (k.phim - phi) * k.inv_dphi;
            T ux = T(0), uy = T(0), uz = T(0), dP = T(0), rho = T(1), om_nu = T(1);
            T fp[3] = {T(0), T(0), T(0)}, ft[3] = {T(0), T(0), T(0)}, gam = T(0);
            T r0g = T(0), jg[3] = {T(0), T(0), T(0)};  // g moments of the node
            int nfault = 0;
            if constexpr (CPL) {
                T gc[3], gq[3];
                // curvature: divergence of the unit normal, same stencil
                const T curv = div3p<T, QX, QP>(nL + ns(z - 1), nL + ns(z), nL + ns(z + 1), qidx);
                grad3p<T, QX>(cL + cs(z - 1), cL + cs(z), cL + cs(z + 1), qidx, gc[0], gc[1],
                              gc[2]);
                grad3p<T, QX>(pL + cs(z - 1), pL + cs(z), pL + cs(z + 1), qidx, gq[0], gq[1],
                              gq[2]);
                const T lam = (phi - k.phi_b) * k.inv_dphi;
                rho = uni_rho ? k.rho_b : k.rho_b + lam * k.drho;
                const T inv_rho = uni_rho ? k.inv_rho_b : rcp_(rho);
                om_nu = uni_nu ? k.omega_nu_b : rcp_(T(3) * (k.nu_b + lam * k.dnu) + T(0.5));
                const T arg = T(1) - c * k.inv_cmax;
                const T sigma = k.sigma0 * (T(1) + k.beta * log_(arg));
                if (!(arg > T(0)) || !(sigma >= T(0))) nfault |= 2;
                const T dsig = -k.sigma0 * k.beta * rcp_(k.c_max - c);
                const T gsg[3] = {dsig * gc[0], dsig * gc[1], dsig * gc[2]};
                const T n3[3] = {nxv, nyv, nzv};
                const T nd = nxv * gsg[0] + nyv * gsg[1] + nzv * gsg[2];
                const T wk = k.ks * gm2;
                const T fe[3] = {k.Fx, k.Fy, k.Fz};
                const T gp[3] = {gpx, gpy, gpz};
                r0g = mom[8 * vol + own];
#pragma unroll
                for (int i = 0; i < 3; ++i) jg[i] = mom[(9 + i) * vol + own];
                T u[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    ft[i] = wk * ((gsg[i] - n3[i] * nd) - sigma * curv * n3[i]) + fe[i];
                    // F_p = -grad psi^, psi^ = P^ - rho cs2, rho linear in phi
                    fp[i] = -(gq[i] - k.dr_cs2 * gp[i]);
                    u[i] = (T(3) * jg[i] + T(0.5) * ft[i]) * inv_rho;
                }
                ux = u[0];
                uy = u[1];
                uz = u[2];
                gam = fp[0] * ux + fp[1] * uy + fp[2] * uz;
                dP = r0g + T(0.5) * gam;
            } else if constexpr (FLOW == FLOW_PRESCRIBED) {
                const T tf = vel_T != 0.0 ? T(cos(M_PI * (double)step / vel_T)) : T(1);
                const T* us = static_cast<const T*>(a.ushape) + uoff;
                ux = us[own] * tf;
                uy = us[vol + own] * tf;
                uz = us[2 * vol + own] * tf;
            }
            if (!isfinite(phi + c + ux + uy + uz + dP)) nfault |= 1;
            // every moment of the node is read, and the prefetched planes are
            // in LDS, before the first population store; the empty asm keeps
            // the compiler from sinking either below the stores
            T mf[4], mh[4], r2[6];
            if constexpr (!FIELDS) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    mf[i] = mom[i * vol + own];
                    mh[i] = mom[(4 + i) * vol + own];
                }
#pragma unroll
                for (int i = 0; i < 6; ++i) r2[i] = CPL ? mom[(12 + i) * vol + own] : T(0);
            }
            flush();
            asm volatile("" ::: "memory");

            if (!col_ok) {
                // nothing to store
            } else if constexpr (FIELDS) {
                fault |= nfault;
                double* o = a.fields_out;
                o[own] = double(phi);
                o[vol + own] = double(c);
                o[2 * vol + own] = double(ux);
                o[3 * vol + own] = double(uy);
                o[4 * vol + own] = double(uz);
                o[5 * vol + own] = CPL ? double(k.P_ref) + double(dP) : 0.0;
            } else {
                fault |= nfault;
                const int lb = 27 * vol * SB;
                char* dstb = static_cast<char*>(a.dst) + soff * SB;
                const int vo = own * SB;
                const int pb = vol * SB;
                uint32_t rs = 0;
                if constexpr (Store<S>::scaled) {
                    const uint32_t key = fmix32((uint32_t)step * 0x9E3779B9u + 0x2504u);
                    rs = cmlb::node_step_seed(node_base + (uint32_t)own, key);
                }
                T t[27];
                // f: phase field
                {
                    const T m0 = mf[0], jx = mf[1], jy = mf[2], jz = mf[3];
                    const T om = k.omega_k, mt = k.M_phi * theta;
                    const T k1x = (T(1) - om) * (jx - ux * phi) + om * mt * nxv;
                    const T k1y = (T(1) - om) * (jy - uy * phi) + om * mt * nyv;
                    const T k1z = (T(1) - om) * (jz - uz * phi) + om * mt * nzv;
                    scalar_dev27<T, MOV>(phi, k1x, k1y, k1z, ux, uy, uz, t);
                    const __amdgpu_buffer_rsrc_t w = make_rsrc(dstb, lb);
#pragma unroll
                    for (int q = 0; q < 27; ++q)
                        Buf<S>::template store<CP>(w, vo, q * pb,
                                                   encode3_add<S>(m0, t[q], k.enc_f, q),
                                                   rs + weyl(q));
                }
                // h: surfactant
                {
                    const T m0 = mh[0], jx = mh[1], jy = mh[2], jz = mh[3];
                    const T om = k.omega_c, mt = k.D_s * theta_c;
                    const T k1x = (T(1) - om) * (jx - ux * c) + om * mt * nxv;
                    const T k1y = (T(1) - om) * (jy - uy * c) + om * mt * nyv;
                    const T k1z = (T(1) - om) * (jz - uz * c) + om * mt * nzv;
                    scalar_dev27<T, MOV>(c, k1x, k1y, k1z, ux, uy, uz, t);
                    const __amdgpu_buffer_rsrc_t w = make_rsrc(dstb + lb, lb);
#pragma unroll
                    for (int q = 0; q < 27; ++q)
                        Buf<S>::template store<CP>(w, vo, q * pb,
                                                   encode3_add<S>(m0, t[q], k.enc_h, q),
                                                   rs + weyl(q));
                }
                // g: flow
                if constexpr (CPL) {
                    const T r0 = r0g;
                    const T j[3] = {jg[0], jg[1], jg[2]};
                    // central second moments of the deviations about u
                    const T u[3] = {ux, uy, uz};
                    T eta2[6];
#pragma unroll
                    for (int i = 0; i < 3; ++i)
                        eta2[i] = r2[i] - T(2) * u[i] * j[i] + u[i] * u[i] * r0;
                    eta2[3] = r2[3] - u[0] * j[1] - u[1] * j[0] + u[0] * u[1] * r0;
                    eta2[4] = r2[4] - u[0] * j[2] - u[2] * j[0] + u[0] * u[2] * r0;
                    eta2[5] = r2[5] - u[1] * j[2] - u[2] * j[1] + u[1] * u[2] * r0;
                    flow_dev27<T>(eta2, dP, rho, ux, uy, uz, fp, ft, gam, k.omega_zeta, om_nu, t);
                    if constexpr (std::is_same_v<S, float>) {
                        // the collision changes the momentum by exactly cs2 F:
                        // raw first moment j + cs2 F, so the central one is
                        // that minus u t0 (no rounding of u in the momentum)
                        const T cs2 = C3<T>::cs2;
                        t[1] = (j[0] + cs2 * ft[0]) - ux * t[0];
                        t[3] = (j[1] + cs2 * ft[1]) - uy * t[0];
                        t[9] = (j[2] + cs2 * ft[2]) - uz * t[0];
                    }
                    inverse27(t, ux, uy, uz);
                    // moving wall: slots of directions pointing into the wall
                    // are pulled back by this node next step; add
                    // 2 rho (e_opp . u_w)
                    T wcorr = T(0);
                    int wdir = 0;
                    if (WALLS) {
                        if (gy == 0) {
                            wdir = -1;
                            wcorr = T(2) * rho * k.u_wall * k.scale_g;
                        }
                        if (gy == ny - 1) {
                            wdir = 1;
                            wcorr = -T(2) * rho * k.u_wall * k.scale_g;
                        }
                    }
                    const __amdgpu_buffer_rsrc_t w = make_rsrc(dstb + 2 * (int64_t)lb, lb);
#pragma unroll
                    for (int q = 0; q < 27; ++q) {
                        T v = encode3<S>(t[q], k.enc_g, q);
                        if (WALLS && wdir != 0 && EYd(q) == wdir) v += wcorr * T(EXd(q));
                        Buf<S>::template store<CP>(w, vo, q * pb, v, rs + weyl(q));
                    }
                }
            }
        }
    }
    if (fault) atomicOr(a.fault + tl.x, fault);
}
// ---------------------------------------------------------------------------
// Initialisation: populations at the central-moment equilibria of given
// fields (FP64), each direction written into the slot it is pulled from.
// ---------------------------------------------------------------------------
struct InitArgs3 {
    void* pop;              // sim's population block
    const SimDev3* sd;
    const double* phi;
    const double* c;
    const double* ux;       // may be null
    const double* uy;
    const double* uz;
    const double* P;        // may be null
    void* ushape;           // prescribed shapes (compute type), may be null
    int32_t flow, walls;
};

// Pull slot of direction a at node (x, y, z): (plane, node index).
__device__ __forceinline__ void pull_slot3(int x, int y, int z, int a, int nx, int ny, int nz,
                                           bool walls, int& pa, int& node) {
    int sx = x - EXd(a), sy = y - EYd(a), sz = z - EZd(a);
    pa = a;
    sx = wrap_coord(sx, nx);
    sz = wrap_coord(sz, nz);
    if (sy < 0 || sy >= ny) {
        if (walls) {
            pa = OPPd(a);
            sx = x;
            sy = y;
            sz = z;
        } else {
            sy = wrap_coord(sy, ny);
        }
    }
    node = (sz * ny + sy) * nx + sx;
}

template <class S, class T>
__device__ __forceinline__ void encode_store(S* base, int64_t idx, double v) {
    base[idx] = S(T(v));
}

template <class S, class T>
__global__ __launch_bounds__(WG3) void k_init3(const InitArgs3 a) {
    const SimDev3* sd = a.sd;
    const int nx = sd->nx, ny = sd->ny, nz = sd->nz, plane = nx * ny, vol = plane * nz;
    const int i = blockIdx.x * WG3 + threadIdx.x;
    if (i >= vol) return;
    const int x = i % nx, y = (i / nx) % ny, z = i / plane;
    const Consts3<double>& k = sd->kd;
    // isotropic gradient of phi with the step's ghost rules
    double g[3] = {0.0, 0.0, 0.0};
    for (int q = 1; q < 27; ++q) {
        const int xx = wrap_coord(x + EXd(q), nx);
        const int yy = a.walls ? mirror_coord(y + EYd(q), ny) : wrap_coord(y + EYd(q), ny);
        const int zz = wrap_coord(z + EZd(q), nz);
        const double v = wgt3<double>(q) * a.phi[(zz * ny + yy) * nx + xx];
        g[0] += EXd(q) * v;
        g[1] += EYd(q) * v;
        g[2] += EZd(q) * v;
    }
    for (int d = 0; d < 3; ++d) g[d] *= 3.0;
    const double inv = 1.0 / (sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) + NORMAL_EPS3);
    const double n3[3] = {g[0] * inv, g[1] * inv, g[2] * inv};
    const double phi = a.phi[i], c = a.c[i];
    const double u[3] = {a.ux ? a.ux[i] : 0.0, a.uy ? a.uy[i] : 0.0, a.uz ? a.uz[i] : 0.0};
    const double theta = k.theta_k * (k.phi_a - phi) * (phi - k.phi_b) * k.inv_dphi;
    const double theta_c = k.thetac_k * c * (k.phim - phi) * k.inv_dphi;
    S* pop = static_cast<S*>(a.pop);
    double t[27];
    // f and h: deviations from the rest distribution about u, then storage
    for (int lat = 0; lat < 2; ++lat) {
        const double s = lat == 0 ? phi : c;
        const double jm = lat == 0 ? k.M_phi * theta : k.D_s * theta_c;
        scalar_dev27<double, true>(s, jm * n3[0], jm * n3[1], jm * n3[2], u[0], u[1], u[2], t);
        const double qref = lat == 0 ? k.qref_f : 0.0;
        const double scale = lat == 0 ? k.scale_f : k.scale_h;
        for (int q = 0; q < 27; ++q) {
            int pa, node;
            pull_slot3(x, y, z, q, nx, ny, nz, a.walls, pa, node);
            const double v = ((s - qref) + t[q] * enc_wgt3<double>(nnz3(q))) * scale;
            encode_store<S, T>(pop, (int64_t)(lat * 27 + pa) * vol + node, v);
        }
    }
    if (a.flow == FLOW_COUPLED) {
        const double lam = (phi - k.phi_b) * k.inv_dphi;
        const double rho = k.rho_b + lam * k.drho;
        const double P = a.P ? a.P[i] : rho * C3<double>::cs2;
        const double dP = P - k.P_ref;
        const double mx[3] = {1.0, -u[0], C3<double>::cs2 + u[0] * u[0]};
        const double my[3] = {1.0, -u[1], C3<double>::cs2 + u[1] * u[1]};
        const double mz[3] = {1.0, -u[2], C3<double>::cs2 + u[2] * u[2]};
        for (int m = 0; m < 27; ++m) {
            const int p = m % 3, q = (m / 3) % 3, r = m / 9;
            const double pm = mx[p] * my[q] * mz[r];
            t[m] = dP * pm + rho * C3<double>::cs2 *
                                 (crest3<double>(p) * crest3<double>(q) * crest3<double>(r) - pm);
        }
        inverse27(t, u[0], u[1], u[2]);
        for (int q = 0; q < 27; ++q) {
            int pa, node;
            pull_slot3(x, y, z, q, nx, ny, nz, a.walls, pa, node);
            encode_store<S, T>(pop, (int64_t)(54 + pa) * vol + node,
                               t[q] * enc_wgt3<double>(nnz3(q)) * k.scale_g);
        }
    }
    if (a.flow == FLOW_PRESCRIBED && a.ushape) {
        T* us = static_cast<T*>(a.ushape);
        us[i] = T(u[0]);
        us[vol + i] = T(u[1]);
        us[2 * vol + i] = T(u[2]);
    }
}

// Decode (dir = 0) or encode (dir = 1) the pre-collision populations of one
// simulation between storage and FP64 host order [lat][27][nz][ny][nx].
template <class S, class T>
__global__ __launch_bounds__(WG3) void k_transfer3(void* pop, const SimDev3* sd, double* host,
                                                   int lattices, int walls, int dir) {
    const int nx = sd->nx, ny = sd->ny, nz = sd->nz, vol = nx * ny * nz;
    const int64_t i = (int64_t)blockIdx.x * WG3 + threadIdx.x;
    if (i >= (int64_t)lattices * 27 * vol) return;
    const int lat = (int)(i / (27 * (int64_t)vol));
    const int q = (int)((i / vol) % 27);
    const int n = (int)(i % vol);
    const int x = n % nx, y = (n / nx) % ny, z = n / (nx * ny);
    int pa, node;
    pull_slot3(x, y, z, q, nx, ny, nz, walls, pa, node);
    const Consts3<double>& k = sd->kd;
    const double scale = lat == 0 ? k.scale_f : (lat == 1 ? k.scale_h : k.scale_g);
    const double qref = lat == 0 ? k.qref_f : (lat == 1 ? 0.0 : k.P_ref);
    const double w = wgt3<double>(q);
    S* p = static_cast<S*>(pop) + (int64_t)(lat * 27 + pa) * vol + node;
    if (dir == 0) {
        host[i] = w * (double(*p) / scale + qref);
    } else {
        *p = S(T((host[i] / w - qref) * scale));
    }
}

// Inventory: FP64 sums of all stored f and h populations (decoded), per
// (y, z) row then over rows in a fixed order.
template <class S>
__global__ __launch_bounds__(WG3) void k_inventory_rows3(const void* pop, const SimDev3* sd,
                                                         double* rows) {
    const int nx = sd->nx, ny = sd->ny, nz = sd->nz, vol = nx * ny * nz;
    const int row = blockIdx.x;  // y + ny z
    const int lat = blockIdx.y;  // 0: f, 1: h
    __shared__ double part[WG3];
    const Consts3<double>& k = sd->kd;
    const double scale = lat == 0 ? k.scale_f : k.scale_h;
    const double qref = lat == 0 ? k.qref_f : 0.0;
    const S* p = static_cast<const S*>(pop) + (int64_t)lat * 27 * vol + (int64_t)row * nx;
    double s = 0.0;
    for (int x = threadIdx.x; x < nx; x += WG3)
        for (int q = 0; q < 27; ++q) s += wgt3<double>(q) * (double(p[(int64_t)q * vol + x]) / scale + qref);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = WG3 / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) rows[lat * ny * nz + row] = part[0];
}

__global__ void k_inventory_final3(const double* rows, int n, double* out) {
    __shared__ double part[WG3];
    for (int lat = 0; lat < 2; ++lat) {
        double s = 0.0;
        for (int i = threadIdx.x; i < n; i += WG3) s += rows[lat * n + i];
        part[threadIdx.x] = s;
        __syncthreads();
        for (int w = WG3 / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[lat] = part[0];
        __syncthreads();
    }
}

}  // namespace cmlb3
