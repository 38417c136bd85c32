// HIP kernels of the coupled central-moment LB step (arXiv 2504.09024) for
// gfx950.  One fused kernel performs a whole time step for every tile of
// every simulation in the context:
//
//   phase 1  pull the 27 (18 without flow) pre-collision populations of the
//            tile's own nodes into registers, q_a(x) = q~_a(x - e_a); zeroth
//            moments phi, c and the pressure deviation P^ - P_ref go to LDS;
//            the halo ring (radius 2 for phi, radius 1 for c and P^) is
//            summed from pulled populations too;
//   phase 2  unit normal n = grad phi/(|grad phi| + eps) on the radius-1
//            ring (coupled flow only, it feeds the curvature);
//   phase 3  per node: interface geometry (theta, theta_c, curvature),
//            Langmuir sigma(c), F_s, F_p, u, P; central-moment collisions
//            of f, h and g; the post-collision populations are stored at the
//            node itself (aligned stores).
//
// Between steps the buffer holds post-collision populations at their own
// node (pull form): reads carry the neighbour shift, writes are aligned,
// which is the faster of the two streaming forms when the working set lives
// in HBM.  At a moving wall (half-way bounce-back) a node pulls the
// directions that would come from behind the wall out of its own opposite
// slots; the momentum correction of g is added when those slots are stored.
#pragma once
#include <type_traits>

#include "lattice.hpp"

namespace cmlb {

constexpr int TX = 64;          // one wavefront spans 64 columns
constexpr int WG = 256;         // threads per workgroup of the auxiliary kernels
constexpr double NORMAL_EPS = 1e-12;

struct StepArgs {
    const void* src;
    void* dst;
    const SimDev* sims;
    const int4* tiles;      // (sim, x0, y0, -)
    int32_t tile_base;
    int32_t ntiles;         // tiles of this launch
    int32_t xcd_remap;      // grid padded to a multiple of 8, remapped per XCD
    int32_t pad_;
    const void* ushape;     // prescribed velocity shapes, compute type
    const int64_t* step_in; // step counter read by this launch
    int64_t* step_out;      // step counter written (n + 1) by workgroup 0
    int32_t* fault;         // per-sim fault bits
    double* fields_out;     // fields mode: [5][ny][nx] (phi, c, ux, uy, P)
};

// Moments of stored scalar-lattice values in storage units.  No FP
// contraction: a node's zeroth moment must carry the same bits in every code
// path that computes it (tile interior and neighbouring tiles' halos).
template <class S, class T>
__device__ __forceinline__ void scalar_moments_nc(const T v[9], T& m0, T& m1, T& m2) {
#pragma clang fp contract(off)
    scalar_moments<T, std::is_same_v<S, float>>(v, m0, m1, m2);
}
template <class S, class T>
__device__ __forceinline__ T scalar_zeroth_nc(const T v[9]) {
#pragma clang fp contract(off)
    T m0, m1, m2;
    scalar_moments<T, std::is_same_v<S, float>>(v, m0, m1, m2);
    return m0;
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

// ---------------------------------------------------------------------------
// Population layout in HBM.  A simulation's populations are kept in runs of
// 64 consecutive nodes of one grid row, the nodes one wavefront covers: run
// r = y * nbx + x / 64 with nbx = ceil(nx / 64).  A run's block holds its
// NL * 9 direction vectors of 64 values one after another, lattice-major:
//     element(lat, q, x, y) = ((r * NL + lat) * 9 + q) * 64 + x mod 64,
// so a wavefront reads and writes one contiguous block per grid row instead
// of NL * 9 planes far apart.  Rows are padded to whole runs (padding slots
// are never read).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t pelem(int lat, int q, int x, int y, int nbx, int nl) {
    return ((((int64_t)y * nbx + (x >> 6)) * nl + lat) * 9 + q) * 64 + (x & 63);
}

// ---------------------------------------------------------------------------
// Pulled loads.  Each lattice has a buffer descriptor that starts at its
// direction 0 in the simulation's first run block, so a value's byte offset
// is r * BLK + a * RUN + (x mod 64) * SB (BLK bytes per run block, RUN per
// direction vector of a run); a simulation's block must fit a 32-bit range.
// On the fast path a node's loads use three vector offsets, the offsets of
// its source columns in row y - 1: vo for x (directions with e_ax = 0), xp
// for x - 1 (e_ax = +1; the previous run for lane 0 of a run, column nx - 1
// at x = 0) and xm for x + 1 (e_ax = -1; the next run for lane 63, column 0
// at x = nx - 1).  Direction a adds a * RUN, a constant the compiler folds
// into the instruction's offset field, and the scalar offset (1 - e_ay) * RB
// (RB bytes per grid row), one of three values.  No offset is negative (a
// raw buffer access whose vector offset wraps below zero reads as out of
// range): the fast path serves rows y >= 1 only.  Near a wall or the y wrap,
// or on grids narrower than a tile plus its halo, the general path folds
// each source (wrap, or the node's own opposite slot at a wall) and
// computes each load's offset on its own.
// ---------------------------------------------------------------------------
template <int SB>
__device__ __forceinline__ void run_offsets(int x, int y, int nx, int nbx, int blk, int& vo,
                                            int& xp, int& xm) {
    const int r = (y - 1) * nbx;
    const int xl = x == 0 ? nx - 1 : x - 1;
    const int xr = x == nx - 1 ? 0 : x + 1;
    vo = (r + (x >> 6)) * blk + (x & 63) * SB;
    xp = (r + (xl >> 6)) * blk + (xl & 63) * SB;
    xm = (r + (xr >> 6)) * blk + (xr & 63) * SB;
}

template <class S, class T>
__device__ __forceinline__ void pull9_inner(__amdgpu_buffer_rsrc_t r, int vo, int xp, int xm,
                                            int row_bytes, T v[9]) {
    constexpr int RUN = 64 * (int)sizeof(S);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const int voff = (EXa(a) > 0 ? xp : (EXa(a) < 0 ? xm : vo)) + a * RUN;
        const int soff = EYa(a) > 0 ? 0 : (EYa(a) == 0 ? row_bytes : 2 * row_bytes);
        v[a] = T(Buf<S>::load(r, voff, soff));
    }
}

template <class S, class T, bool WALLS>
__device__ __forceinline__ void pull9_edge(__amdgpu_buffer_rsrc_t r, int lx, int ly, int nx,
                                           int ny, int nbx, int blk, T v[9]) {
    constexpr int RUN = 64 * (int)sizeof(S);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        int sx = lx - EXa(a), sy = ly - EYa(a), pa = a;
        if (sx < 0) sx += nx;
        else if (sx >= nx) sx -= nx;
        if (sy < 0 || sy >= ny) {
            if (WALLS) {
                pa = OPPa(a);
                sx = lx;
                sy = ly;
            } else {
                sy = sy < 0 ? sy + ny : sy - ny;
            }
        }
        // the direction varies per lane here (bounce-back), so it goes into
        // the vector offset
        v[a] = T(Buf<S>::load(r, (sy * nbx + (sx >> 6)) * blk + pa * RUN + (sx & 63) * (int)sizeof(S),
                              0));
    }
}

// stored g values -> deviations d_a = w_a s_a / scale.  FP32 storage (scale
// 1): w_a s_a as (9 w_a) s_a / 9, 9 w_a in {4, 1, 1/4} exact, with a
// correctly rounded division, so the moments carry no common weight bias.
template <class S, class T, class KP>
__device__ __forceinline__ void to_dev(T v[9], const KP& k) {
#pragma clang fp contract(off)
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        if constexpr (std::is_same_v<S, float>) {
            v[a] = div_const<9>((a == 0 ? T(4) : (a < 5 ? T(1) : T(0.25))) * v[a]);
        } else if constexpr (Store<S>::scaled) {
            // one product with w_a / scale_g (scale_g a power of two)
            v[a] = v[a] * (a == 0 ? k.wdec0 : (a < 5 ? k.wdec1 : k.wdec5));
        } else {
            v[a] = wgt<T>(a) * v[a];
        }
    }
}

// Slot from which node (x, y) pulls direction a: (direction plane, source
// column, source row).
__device__ __forceinline__ void pull_slot(int x, int y, int a, int nx, int ny, bool walls,
                                          int& plane_a, int& sx, int& sy) {
    sx = x - EXa(a);
    sy = y - EYa(a);
    plane_a = a;
    if (sx < 0) sx += nx;
    else if (sx >= nx) sx -= nx;
    if (sy < 0 || sy >= ny) {
        if (walls) {
            plane_a = OPPa(a);
            sx = x;
            sy = y;
        } else {
            sy = sy < 0 ? sy + ny : sy - ny;
        }
    }
}

template <class T>
__device__ __forceinline__ const PhysConsts<T>& consts(const SimDev* sd);
template <>
__device__ __forceinline__ const PhysConsts<double>& consts<double>(const SimDev* sd) {
    return sd->kd;
}
template <>
__device__ __forceinline__ const PhysConsts<float>& consts<float>(const SimDev* sd) {
    return sd->kf;
}


// ---------------------------------------------------------------------------
// The fused step kernel.  FIELDS = true evaluates phases 1-3 up to the
// macroscopic fields and writes them instead of colliding.
// ---------------------------------------------------------------------------
// Launch shape: NW waves per workgroup, NPT rows per thread, tile 64 x NW*NPT.
// At most 128 VGPRs for FP32 storage so that four waves fit per SIMD.
template <class T, int NW>
struct Occupancy {
    static constexpr int waves_per_eu = sizeof(T) == 4 ? 4 : (NW >= 8 ? 2 : 2);
};

// NTS: population stores non-temporal (for lattices too large to stay in the
// last-level cache between steps).
// WX: wavefronts across x, so a tile is 64*WX columns by (NW/WX)*NPT rows;
// wider tiles share fewer partly-used cache lines with their x neighbours.
template <class S, class T, int FLOW, bool WALLS, int NW, int NPT, bool FIELDS, bool NTS, int WX>
__global__ __launch_bounds__(NW * 64, (Occupancy<T, NW>::waves_per_eu)) void k_step(const StepArgs a) {
    static_assert(NW % WX == 0, "waves must tile the width");
    constexpr int CP = NTS ? CPOL_NT : 0;
    constexpr int NT = NW * 64;
    constexpr bool CPL = FLOW == FLOW_COUPLED;
    constexpr bool MOV = FLOW != FLOW_NONE;
    constexpr int TW = TX * WX;
    constexpr int TY = (NW / WX) * NPT;
    constexpr int PW = TW + 4, PH = TY + 4;  // phi region (radius 2)
    constexpr int QW = TW + 2, QH = TY + 2;  // c, P^, n region (radius 1)
    constexpr int RING = 4 * PW + 4 * TY;
    constexpr int SB = sizeof(S);
    __shared__ T phiL[PH * PW];
    __shared__ T cL[QH * QW];
    __shared__ T pL[CPL ? QH * QW : 1];
    __shared__ T nxL[CPL ? QH * QW : 1];
    __shared__ T nyL[CPL ? QH * QW : 1];

    // Workgroups are dispatched round-robin over the 8 XCDs (each with its
    // own L2): give XCD k the contiguous tile range [k*per, (k+1)*per) so that
    // neighbouring tiles, whose rows and halos overlap, share one L2.
    int tix = blockIdx.x;
    if (a.xcd_remap) {
        const int per = (int)gridDim.x >> 3;
        tix = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
        if (tix >= a.ntiles) return;
    }
    const int4 tl = a.tiles[a.tile_base + tix];
    const SimDev* sd = a.sims + tl.x;
    // FP32: the simulation's constants by value, read once into scalar
    // registers before any store (a population store could alias the table
    // for all the compiler knows, and a reload after a store would wait for
    // the store).  FP64 keeps reading them on use: twice the scalar
    // registers would spill.
    using KRef = std::conditional_t<(sizeof(T) > 4), const PhysConsts<T>&, const PhysConsts<T>>;
    KRef k = consts<T>(sd);
    const int nx = sd->nx, ny = sd->ny;
    const uint32_t node_base = sd->node_base;
    const int64_t ushape_off = sd->ushape_off;
    const int x0 = tl.y, y0 = tl.z;
    const int plane = nx * ny;
    constexpr int NL = CPL ? 3 : 2;     // lattices
    constexpr int RUN = 64 * SB;        // bytes per direction vector of a run
    constexpr int BLK = NL * 9 * RUN;   // bytes per run block
    const int nbx = (nx + 63) >> 6;     // runs per grid row
    const int RB = nbx * BLK;           // bytes per grid row
    const char* srcb = static_cast<const char*>(a.src) + sd->off * SB;
    const int64_t step = *a.step_in;
    // tile, its radius-2 halo and their pull sources clear of the walls (or
    // of the y wrap), on a grid at least a tile and its halo wide: x wraps
    // per lane on the fast path
    const bool inner = y0 >= 3 && y0 + TY + 3 <= ny && nx >= TW + 3;
    const int sim_bytes = ny * RB;
    const __amdgpu_buffer_rsrc_t rF = make_rsrc(srcb, sim_bytes);
    const __amdgpu_buffer_rsrc_t rH = make_rsrc(srcb + 9 * RUN, sim_bytes - 9 * RUN);
    const __amdgpu_buffer_rsrc_t rG =
        make_rsrc(srcb + (CPL ? 18 * RUN : 0), sim_bytes - (CPL ? 18 * RUN : 0));

    const int tid = threadIdx.x;
    static_assert((WX & (WX - 1)) == 0, "WX must be a power of two");
    const int wave = tid / TW;        // row block of this wavefront
    const int lane = tid & (TW - 1);  // column within the tile
    const int gx = x0 + lane;
    // lanes past the right edge of a ragged tile load the wrapped column;
    // they store nothing
    const int lx = inner ? (gx < nx ? gx : gx - nx) : wrap_coord(gx, nx);

    // ---------------- phase 1: own nodes -----------------------------------
    // FP32 storage with non-temporal stores (working sets beyond the
    // Infinity Cache): the wave issues its own pulls at raised priority, so a
    // wave entering the step gets its loads out ahead of the arithmetic of
    // the other waves on its SIMD (64-drop batch: +4%).  The same costs
    // 8-10% in FP16 or FP64, where the arithmetic is the scarcer resource,
    // and 2.7% on the cache-resident 1024x512 drop (default stores), so
    // those keep the default priority.
    constexpr bool LOAD_PRIO = std::is_same_v<S, float> && NTS;
    if constexpr (LOAD_PRIO) __builtin_amdgcn_s_setprio(2);
    T qf[NPT][9], qh[NPT][9], qg[CPL ? NPT : 1][9];
    T phv[NPT], cv[NPT], phn[NPT], chn[NPT], jfx[NPT], jfy[NPT], jhx[NPT], jhy[NPT];
    Raw6<T> mg[CPL ? NPT : 1];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int iy = wave * NPT + j;
        const int gy = y0 + iy;
        if (inner) {
            int vo, xp, xm;
            run_offsets<SB>(lx, gy, nx, nbx, BLK, vo, xp, xm);
            pull9_inner<S, T>(rF, vo, xp, xm, RB, qf[j]);
            pull9_inner<S, T>(rH, vo, xp, xm, RB, qh[j]);
            if constexpr (CPL) pull9_inner<S, T>(rG, vo, xp, xm, RB, qg[j]);
        } else {
            const int ly = WALLS ? mirror_coord(gy, ny) : wrap_coord(gy, ny);
            pull9_edge<S, T, WALLS>(rF, lx, ly, nx, ny, nbx, BLK, qf[j]);
            pull9_edge<S, T, WALLS>(rH, lx, ly, nx, ny, nbx, BLK, qh[j]);
            if constexpr (CPL) pull9_edge<S, T, WALLS>(rG, lx, ly, nx, ny, nbx, BLK, qg[j]);
        }
    }
    if constexpr (LOAD_PRIO) __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int iy = wave * NPT + j;
        scalar_moments_nc<S>(qf[j], phn[j], jfx[j], jfy[j]);
        scalar_moments_nc<S>(qh[j], chn[j], jhx[j], jhy[j]);
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
            to_dev<S, T>(qg[j], k);
            mg[j] = moments6_nc(qg[j]);
            pL[(iy + 1) * QW + lane + 1] = mg[j].m0;
        }
    }
    // ---------------- phase 1b: halo ring ----------------------------------
    // a compile-time trip count: with a runtime loop the ring's values and
    // the own nodes' populations outgrow 128 VGPRs in 128-wide tiles (two
    // ring nodes per thread) and spill
    constexpr int RITER = (RING + NT - 1) / NT;
#pragma unroll
    for (int it = 0; it < RITER; ++it) {
        const int i = tid + it * NT;
        if (i >= RING) break;
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
        int hx = x0 - 2 + rx, hy = y0 - 2 + ry;
        const bool r1 = ry >= 1 && ry <= PH - 2 && rx >= 1 && rx <= PW - 2;
        const int qi = (ry - 1) * QW + rx - 1;
        T q[9];
        if (inner) {
            hx = hx < 0 ? hx + nx : (hx >= nx ? hx - nx : hx);
            int vo, xp, xm;
            run_offsets<SB>(hx, hy, nx, nbx, BLK, vo, xp, xm);
            pull9_inner<S, T>(rF, vo, xp, xm, RB, q);
            phiL[ry * PW + rx] = scalar_zeroth_nc<S>(q) * k.inv_f + k.qref_f;
            if (r1) {
                pull9_inner<S, T>(rH, vo, xp, xm, RB, q);
                cL[qi] = scalar_zeroth_nc<S>(q) * k.inv_h;
                if constexpr (CPL) {
                    pull9_inner<S, T>(rG, vo, xp, xm, RB, q);
                    to_dev<S, T>(q, k);
                    pL[qi] = zeroth(q);
                }
            }
        } else {
            hx = wrap_coord(hx, nx);
            hy = WALLS ? mirror_coord(hy, ny) : wrap_coord(hy, ny);
            pull9_edge<S, T, WALLS>(rF, hx, hy, nx, ny, nbx, BLK, q);
            phiL[ry * PW + rx] = scalar_zeroth_nc<S>(q) * k.inv_f + k.qref_f;
            if (r1) {
                pull9_edge<S, T, WALLS>(rH, hx, hy, nx, ny, nbx, BLK, q);
                cL[qi] = scalar_zeroth_nc<S>(q) * k.inv_h;
                if constexpr (CPL) {
                    pull9_edge<S, T, WALLS>(rG, hx, hy, nx, ny, nbx, BLK, q);
                    to_dev<S, T>(q, k);
                    pL[qi] = zeroth(q);
                }
            }
        }
    }
    __syncthreads();

    // ---------------- phase 2: unit normal on the radius-1 region ----------
    if constexpr (CPL) {
        for (int i = tid; i < QH * QW; i += NT) {
            const int qy = i / QW, qx = i - qy * QW;
            T gxv, gyv;
            lds_grad<T, PW>(phiL, (qy + 1) * PW + qx + 1, gxv, gyv);
            const T inv = rcp_(sqrt_(gxv * gxv + gyv * gyv) + T(NORMAL_EPS));
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
    char* dstb = static_cast<char*>(a.dst) + sd->off * SB;
    const __amdgpu_buffer_rsrc_t wF = make_rsrc(dstb, sim_bytes);
    const __amdgpu_buffer_rsrc_t wH = make_rsrc(dstb + 9 * RUN, sim_bytes - 9 * RUN);
    const __amdgpu_buffer_rsrc_t wG =
        make_rsrc(dstb + (CPL ? 18 * RUN : 0), sim_bytes - (CPL ? 18 * RUN : 0));
    const bool urho = sd->uniform_rho, unu = sd->uniform_nu;
    const uint32_t step_key = fmix32((uint32_t)step * 0x9E3779B9u + 0x2504u);
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
            const T inv = rcp_(sqrt_(gm2) + T(NORMAL_EPS));
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
            rho = urho ? k.rho_b : k.rho_b + lam * k.drho;
            const T inv_rho = urho ? k.inv_rho_b : rcp_(rho);
            omega_nu = unu ? k.omega_nu_b : rcp_(T(3) * (k.nu_b + lam * k.dnu) + T(0.5));
            const T arg = T(1) - c * k.inv_cmax;
            const T sigma = k.sigma0 * (T(1) + k.beta * log_(arg));
            if (valid && (!(arg > T(0)) || !(sigma >= T(0)))) fault |= 2;
            const T dsig = -k.sigma0 * k.beta * rcp_(k.c_max - c);
            const T gsx = dsig * gcx, gsy = dsig * gcy;
            const T nd = nxv * gsx + nyv * gsy;
            const T tsx = gsx - nxv * nd, tsy = gsy - nyv * nd;
            const T wk = k.ks * gm2;
            ftx = wk * (tsx - sigma * curv * nxv) + k.Fx;
            fty = wk * (tsy - sigma * curv * nyv) + k.Fy;
            // F_p = -grad psi^, psi^ = P^ - rho cs2, rho linear in phi
            fpx = -(gqx - k.dr_cs2 * gpx);
            fpy = -(gqy - k.dr_cs2 * gpy);
            if constexpr (sizeof(T) == 4) {
                // the collision re-encodes the momentum as u (T00 - psi),
                // T00 - psi = fl(rho cs2) + ..., with cs2 rounded to FP32
                // (1 + 3e-8 times 1/3): the velocity divides by that same
                // product (quotient corrected by one residual step), where
                // 3 m1 / rho would grow u by 3e-8 every step
                const T crho = rho * K<T>::cs2;
                const T ic = rcp_(crho);
                const T q0x = mg[j].m1 * ic, q0y = mg[j].m2 * ic;
                const T qx = fmaf(fmaf(-q0x, crho, mg[j].m1), ic, q0x);
                const T qy = fmaf(fmaf(-q0y, crho, mg[j].m2), ic, q0y);
                ux = qx + T(0.5) * ftx * inv_rho;
                uy = qy + T(0.5) * fty * inv_rho;
            } else {
                ux = (T(3) * mg[j].m1 + T(0.5) * ftx) * inv_rho;
                uy = (T(3) * mg[j].m2 + T(0.5) * fty) * inv_rho;
            }
            gam = fpx * ux + fpy * uy;
            dP = mg[j].m0 + T(0.5) * gam;
            psi = dP + (k.P_ref - rho * K<T>::cs2);
        } else if constexpr (FLOW == FLOW_PRESCRIBED) {
            const T* us = static_cast<const T*>(a.ushape) + ushape_off;
            const int ni = gy < ny ? gy * nx + lx : lx;
            ux = us[ni] * tf;
            uy = us[plane + ni] * tf;
        }
        if (valid && !isfinite(phi + c + ux + uy + dP)) fault |= 1;

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
            T r[9];
            {
                const T k1 = (T(1) - k.omega_k) * (jfx[j] - ux * phi) + k.omega_k * k.M_phi * theta * nxv;
                const T k2 = (T(1) - k.omega_k) * (jfy[j] - uy * phi) + k.omega_k * k.M_phi * theta * nyv;
                scalar_post_dev<T, MOV>(phi, k1, k2, ux, uy, r);
                pinv_dev_add(r, k.scale_f, phn[j], qf[j]);
            }
            // h: interface-bound surfactant (Sec. 3)
            {
                const T k1 = (T(1) - k.omega_c) * (jhx[j] - ux * c) + k.omega_c * k.D_s * theta_c * nxv;
                const T k2 = (T(1) - k.omega_c) * (jhy[j] - uy * c) + k.omega_c * k.D_s * theta_c * nyv;
                scalar_post_dev<T, MOV>(c, k1, k2, ux, uy, r);
                pinv_dev_add(r, k.scale_h, chn[j], qh[j]);
            }
            // g: two-fluid flow (App. D)
            if constexpr (CPL) {
                T t[9];
                const T P_hat = k.P_ref + mg[j].m0;
                flow_collide(mg[j], ux, uy, dP, psi, P_hat, fpx, fpy, ftx, fty, gam,
                             k.omega_zeta, omega_nu, t);
                flow_post_raw(t, ux, uy, k.P_ref, r);
                if constexpr (std::is_same_v<S, float>) {
                    // FP32 storage.  The collision changes the momentum by
                    // exactly cs2 F (u (rho cs2 + gam/2) + (cs2 F - u gam)/2
                    // with rho cs2 u = m1 + cs2 F/2): taken as that sum, no
                    // rounding of u enters it.  The third-order moments carry
                    // the rest value u rho_b/9 (kappa_xx of the rest state
                    // times u); formed as u (t + cs2 P_ref) it would take the
                    // 7.45e-9 bias of the rounded 1/9 every step, and these
                    // two moments decide the momentum a moving wall hands to
                    // the fluid (a steady slip of 1e-5 of the wall speed in
                    // the 1024 x 512 shear drop).
                    const T uxuy = ux * uy, ux2 = ux * ux, uy2 = uy * uy;
                    const T T00 = t[0] + k.P_ref;
                    r[1] = mg[j].m1 + K<T>::cs2 * ftx;
                    r[2] = mg[j].m2 + K<T>::cs2 * fty;
                    r[6] = ux2 * uy * T00 + T(2) * uxuy * t[1] + ux2 * t[2] + uy * t[3] +
                           div_const<9>(uy * k.rho_b) + T(2) * ux * t[5] + t[6];
                    r[7] = ux * uy2 * T00 + uy2 * t[1] + T(2) * uxuy * t[2] + ux * t[4] +
                           div_const<9>(ux * k.rho_b) + T(2) * uy * t[5] + t[7];
                } else if constexpr (sizeof(T) == 4) {
                    // first raw moments u (T00 - psi) + s1/2 with
                    // T00 - psi = fl(rho cs2) + gam/2 taken directly: T00 =
                    // P_ref + t0 in FP32 rounds the pressure deviation to
                    // 3e-8, the same every step at a quasi-steady node
                    const T crho = rho * K<T>::cs2;
                    const T mom = crho + T(0.5) * gam;
                    r[1] = ux * mom + T(0.5) * (K<T>::cs2 * ftx - ux * gam);
                    r[2] = uy * mom + T(0.5) * (K<T>::cs2 * fty - uy * gam);
                }
                if constexpr (std::is_same_v<S, float>) {
                    // FP32 storage: the map back to populations in FP64, so
                    // the stored values carry the one rounding of the store.
                    // The FP32 sums of this map round the same way at a
                    // quasi-steady node every step; the momentum they leave
                    // acts as a small steady force (FP32 against FP64, the
                    // velocity of the 1024 x 512 shear drop at Ca = 0.5 after
                    // 5000 steps: 6.0e-6 with this map in FP32, 7.9e-7 in FP64).
                    pinv_dev_wide(r, k.scale_g, qg[j]);
                } else {
                    pinv_dev(r, k.scale_g, qg[j]);
                }
            }
            if (valid) {
                const int own = gy * nx + gx;
                const int vo = (gy * nbx + (gx >> 6)) * BLK + (gx & 63) * SB;
                uint32_t rs = 0;
                if constexpr (Store<S>::scaled) rs = node_step_seed(node_base + (uint32_t)own, step_key);
                // moving wall: the slots of directions pointing into the wall
                // are pulled back by this node next step (half-way
                // bounce-back); g carries the momentum correction
                // 2 rho (e_opp . u_w) in storage units, u_w = -+u_wall.
                T wcorr = T(0);
                int wdir = 0;
                if (WALLS) {
                    if (gy == 0) { wdir = -1; wcorr = T(2) * rho * k.u_wall * k.scale_g; }
                    if (gy == ny - 1) { wdir = 1; wcorr = -T(2) * rho * k.u_wall * k.scale_g; }
                }
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    const int off = vo + q * RUN;
                    const uint32_t rq = rs + weyl(q);
                    Buf<S>::template store<CP>(wF, off, 0, qf[j][q], rq);
                    Buf<S>::template store<CP>(wH, off, 0, qh[j][q], rq);
                    if constexpr (CPL) {
                        T v = qg[j][q];
                        if (WALLS && wdir != 0 && EYa(q) == wdir) v += wcorr * T(EXa(q));
                        Buf<S>::template store<CP>(wG, off, 0, v, rq);
                    }
                }
            }
        }
    }
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

// Each node computes its pre-collision equilibria and writes each direction
// into the slot it will pull that direction from, so the first step sees
// exactly these populations (every slot has one writer).
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
    double r[9], sf[9], sh[9], sg[9];
    scalar_post_dev<double, true>(phi, sd->M_phi * theta * nxv, sd->M_phi * theta * nyv, ux, uy, r);
    pinv_dev(r, sd->scale_f, sf);
    const double phin = (phi - sd->qref_f) * sd->scale_f;
    scalar_post_dev<double, true>(c, sd->D_s * theta_c * nxv, sd->D_s * theta_c * nyv, ux, uy, r);
    pinv_dev(r, sd->scale_h, sh);
    const double chn = c * sd->scale_h;
    const bool cpl = a.flow == FLOW_COUPLED;
    if (cpl) {
        const double lam = (phi - sd->phi_b) * sd->inv_dphi;
        const double rho = sd->rho_b + lam * sd->drho;
        const double P = a.P ? a.P[i] : rho * K<double>::cs2;
        const double psi = P - rho * K<double>::cs2;
        double t[9];
        flow_eq_dev(P - sd->P_ref, psi, ux, uy, t);
        flow_post_raw(t, ux, uy, sd->P_ref, r);
        pinv_encode(r, sd->scale_g, 0.0, sg);
    }
    const int nl = cpl ? 3 : 2, nbx = (nx + 63) >> 6;
    for (int q = 0; q < 9; ++q) {
        int pq, sx, sy;
        pull_slot(x, y, q, nx, ny, a.walls != 0, pq, sx, sy);
        pop[pelem(0, pq, sx, sy, nbx, nl)] = S(phin + sf[q]);
        pop[pelem(1, pq, sx, sy, nbx, nl)] = S(chn + sh[q]);
        if (cpl) pop[pelem(2, pq, sx, sy, nbx, nl)] = S(sg[q]);
    }
    if (a.flow == FLOW_PRESCRIBED && a.ushape) {
        T* us = static_cast<T*>(a.ushape);
        us[i] = T(ux);
        us[plane + i] = T(uy);
    }
}

// ---------------------------------------------------------------------------
// Population transfer: the pre-collision populations of each node (pulled
// from their slots) to plain FP64, and back.
// ---------------------------------------------------------------------------
template <class S>
__global__ __launch_bounds__(WG) void k_decode(const void* pop, const SimDev* sd, int nlat,
                                               int walls, double* out) {
    const int nx = sd->nx, ny = sd->ny, plane = nx * ny;
    const int64_t total = (int64_t)nlat * 9 * plane;
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= total) return;
    const int lat = (int)(i / (9 * (int64_t)plane));
    const int q = (int)((i / plane) % 9);
    const int n = (int)(i % plane);
    int pq, sx, sy;
    pull_slot(n % nx, n / nx, q, nx, ny, walls != 0, pq, sx, sy);
    const double s =
        double(static_cast<const S*>(pop)[pelem(lat, pq, sx, sy, (nx + 63) >> 6, nlat)]);
    const double w = wgt<double>(q);
    const double scale = lat == 0 ? sd->scale_f : (lat == 1 ? sd->scale_h : sd->scale_g);
    const double qref = lat == 0 ? sd->qref_f : (lat == 1 ? 0.0 : sd->P_ref);
    out[i] = w * (s / scale + qref);
}

template <class S>
__global__ __launch_bounds__(WG) void k_encode(void* pop, const SimDev* sd, int nlat, int walls,
                                               const double* in) {
    const int nx = sd->nx, ny = sd->ny, plane = nx * ny;
    const int64_t total = (int64_t)nlat * 9 * plane;
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= total) return;
    const int lat = (int)(i / (9 * (int64_t)plane));
    const int q = (int)((i / plane) % 9);
    const int n = (int)(i % plane);
    int pq, sx, sy;
    pull_slot(n % nx, n / nx, q, nx, ny, walls != 0, pq, sx, sy);
    const double scale = lat == 0 ? sd->scale_f : (lat == 1 ? sd->scale_h : sd->scale_g);
    const double qref = lat == 0 ? sd->qref_f : (lat == 1 ? 0.0 : sd->P_ref);
    const double s = (in[i] * inv_wgt<double>(q) - qref) * scale;
    static_cast<S*>(pop)[pelem(lat, pq, sx, sy, (nx + 63) >> 6, nlat)] = S(s);
}

// ---------------------------------------------------------------------------
// Inventories: FP64 totals of phi and c for the simulations [first, first+n)
// of a context in two launches.  Stage 1 has one workgroup per (simulation,
// row), workgroup index = (sim - first) * max_ny + row: each thread sums its
// columns in order, then a fixed butterfly over the wave and a fixed order
// over the waves give the row's partial, stored at index row0 - row_base + y.
// Stage 2 has one workgroup per simulation, whose first thread adds that
// simulation's row partials in row order.  The order of every addition is
// fixed, so a total does not depend on the step kernel's tiling, on which
// other simulations share the launch, or on the buffer the partials go to.
// ---------------------------------------------------------------------------
template <class S>
__global__ __launch_bounds__(WG) void k_inventory_rows(const void* pop, const SimDev* sims,
                                                       int nl, int first, int max_ny,
                                                       int row_base, double* rows) {
    const SimDev* sd = sims + first + (int)(blockIdx.x / max_ny);
    const int nx = sd->nx, ny = sd->ny;
    const int y = (int)(blockIdx.x % max_ny);
    if (y >= ny) return;
    const S* p = static_cast<const S*>(pop) + sd->off;
    const double inv_f = 1.0 / sd->scale_f, inv_h = 1.0 / sd->scale_h, qref = sd->qref_f;
    const int nbx = (nx + 63) >> 6;
    double sf = 0.0, sh = 0.0;
    for (int x = threadIdx.x; x < nx; x += WG) {
        double vf = 0.0, vh = 0.0;
        for (int q = 0; q < 9; ++q) {
            const double w = wgt<double>(q);
            vf += w * (double(p[pelem(0, q, x, y, nbx, nl)]) * inv_f + qref);
            vh += w * (double(p[pelem(1, q, x, y, nbx, nl)]) * inv_h);
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
        const int r = sd->row0 - row_base + y;
        rows[2 * r] = a;
        rows[2 * r + 1] = b;
    }
}

__global__ __launch_bounds__(WG) void k_inventory_final(const double* rows, const SimDev* sims,
                                                        int first, int row_base, double* out) {
    // one workgroup per simulation: chunks of the row partials are staged in
    // LDS by all threads, then one thread adds them in row order
    const SimDev* sd = sims + first + blockIdx.x;
    const int r0 = sd->row0 - row_base, ny = sd->ny;
    __shared__ double buf[2 * WG];
    double a = 0.0, b = 0.0;
    for (int y0 = 0; y0 < ny; y0 += WG) {
        const int n = min(WG, ny - y0);
        if ((int)threadIdx.x < n) {
            buf[2 * threadIdx.x] = rows[2 * (r0 + y0 + threadIdx.x)];
            buf[2 * threadIdx.x + 1] = rows[2 * (r0 + y0 + threadIdx.x) + 1];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int y = 0; y < n; ++y) {
                a += buf[2 * y];
                b += buf[2 * y + 1];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = a;
        out[2 * blockIdx.x + 1] = b;
    }
}

}  // namespace cmlb
