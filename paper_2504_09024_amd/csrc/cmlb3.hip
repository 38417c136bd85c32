// Host runtime of the 3D (D3Q27) coupled central-moment LB library: the C ABI
// of include/cmlb3.h.  Device work is in kernels3.hpp; a step is the moments
// launch followed by the collision launch, over tile tables that cover every
// simulation of the context.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/cmlb3.h"
#include "kernels3.hpp"

using namespace cmlb3;

namespace {

constexpr int GRAPH_STEPS3 = 16;  // steps per graph (even: the graph ends on its start parity)
// collision columns 64 x ty nodes (ty waves) marching through zs planes;
// the field read-out uses 64 x 4 columns of 8 planes
struct Shape3 {
    int ty, zs;
};
const Shape3 SHAPES3[] = {{4, 16}, {4, 8}, {8, 16}, {8, 8}, {4, 4}};
constexpr int N_SHAPES3 = sizeof(SHAPES3) / sizeof(Shape3);
constexpr int FTY = 4, FZS = 8;
// fastest measured on the 256 x 128 x 128 coupled drop: FP32 64 x 8 columns
// of 16 planes; FP16 and FP64 64 x 4 columns of 8 planes (FP64 at 64 x 8
// would spill registers to memory)
Shape3 default_shape3(int prec) { return prec == CMLB_FP32 ? Shape3{8, 16} : Shape3{4, 8}; }

size_t sbytes(int prec) { return prec == CMLB_FP64 ? 8 : (prec == CMLB_FP32 ? 4 : 2); }
double omega3(double coeff) { return 1.0 / (coeff * 3.0 + 0.5); }
bool rate_ok3(double w) { return std::isfinite(w) && w > 0.0 && w < 2.0; }
double pow2_floor3(double v) { return std::ldexp(1.0, (int)std::floor(std::log2(v))); }

// double-precision description of one simulation (host side)
struct Desc3 {
    double scale_f, scale_h, scale_g, qref_f, P_ref;
};

template <class T>
void fill3(Consts3<T>& k, const cmlb3_sim_params& p, const Desc3& d, int walls) {
    const double dphi = p.phi_a - p.phi_b, phio = 0.5 * dphi;
    k.inv_f = T(1.0 / d.scale_f);
    k.qref_f = T(d.qref_f);
    k.scale_f = T(d.scale_f);
    k.inv_h = T(1.0 / d.scale_h);
    k.scale_h = T(d.scale_h);
    k.inv_g = T(1.0 / d.scale_g);
    k.scale_g = T(d.scale_g);
    // the weights rounded to T as on the device, then scaled by the power of
    // two 1/scale_g (exact)
    const T wn[4] = {T(8) / T(27), T(2) / T(27), T(1) / T(54), T(1) / T(216)};
    for (int n = 0; n < 4; ++n) k.wdec3[n] = T(wn[n] * T(1.0 / d.scale_g));
    k.phi_a = T(p.phi_a);
    k.phi_b = T(p.phi_b);
    k.inv_dphi = T(1.0 / dphi);
    k.phim = T(0.5 * (p.phi_a + p.phi_b));
    k.theta_k = T(4.0 / p.W);
    k.thetac_k = T(8.0 / p.W);
    k.M_phi = T(p.M_phi);
    k.D_s = T(p.D_s);
    k.omega_k = T(omega3(p.M_phi));
    k.omega_c = T(omega3(p.D_s));
    k.rho_b = T(p.rho_b);
    k.drho = T(p.rho_a - p.rho_b);
    k.nu_b = T(p.nu_b);
    k.dnu = T(p.nu_a - p.nu_b);
    k.inv_rho_b = T(1.0 / p.rho_b);
    k.omega_nu_b = T(omega3(p.nu_b));
    k.omega_zeta = T(p.omega_zeta);
    k.sigma0 = T(p.sigma0);
    k.beta = T(p.beta);
    k.c_max = T(p.c_max);
    k.inv_cmax = T(p.c_max != 0.0 ? 1.0 / p.c_max : 0.0);
    k.ks = T(3.0 * p.W / (8.0 * phio * phio));
    k.u_wall = T(walls ? p.u_wall : 0.0);
    k.Fx = T(p.F_ext_x);
    k.Fy = T(p.F_ext_y);
    k.Fz = T(p.F_ext_z);
    k.P_ref = T(d.P_ref);
    k.dr_cs2 = T((p.rho_a - p.rho_b) / dphi / 3.0);
    for (int n = 0; n < 4; ++n) {
        // 1/w_a / 2^n = (27/8) 2^n, times the power-of-two storage scale
        k.enc_f[n] = T(d.scale_f * 3.375 * (1 << n));
        k.enc_h[n] = T(d.scale_h * 3.375 * (1 << n));
        k.enc_g[n] = T(d.scale_g * 3.375 * (1 << n));
    }
}

}  // namespace

struct cmlb3_ctx {
    int n_sims = 0, prec = 0, flow = 0, walls = 0, nlat = 2;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<cmlb3_sim_params> params;
    std::vector<SimDev3> sims;
    std::vector<char> inited;
    int64_t pop_elems = 0, mom_elems = 0, ushape_elems = 0, max_vol = 0, max_rows = 0;
    void* pop[2] = {nullptr, nullptr};
    void* mom = nullptr;
    void* ushape = nullptr;
    SimDev3* d_sims = nullptr;
    int4* d_mtiles = nullptr;
    int4* d_ctiles = nullptr;
    int4* d_ftiles = nullptr;
    int n_mtiles = 0, n_ctiles = 0;
    int cty = 4, czs = 16;          // collision column shape
    int store_policy = 0;           // 0 auto, 1 default stores, 2 non-temporal stores
    int64_t pop_bytes = 0;
    std::vector<int> ftile0, fntiles;
    int64_t* d_step = nullptr;
    int32_t* d_fault = nullptr;
    double* d_rows = nullptr;
    double* d_inv = nullptr;
    int cur = 0;
    int64_t step = 0;
    int use_graph = 1;
    bool fault_seen = false;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    std::string err;
};

namespace {

int fail3(cmlb3_ctx* c, int code, const char* fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIP3(ctx, expr)                                                                      \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail3((ctx), CMLB_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

void drop_graphs3(cmlb3_ctx* c) {
    for (int i = 0; i < 2; ++i) {
        if (c->gexec[i]) (void)hipGraphExecDestroy(c->gexec[i]);
        if (c->graph[i]) (void)hipGraphDestroy(c->graph[i]);
        c->gexec[i] = nullptr;
        c->graph[i] = nullptr;
    }
}

void release3(cmlb3_ctx* c) {
    drop_graphs3(c);
    (void)hipFree(c->pop[0]);
    (void)hipFree(c->pop[1]);
    (void)hipFree(c->mom);
    (void)hipFree(c->ushape);
    (void)hipFree(c->d_sims);
    (void)hipFree(c->d_mtiles);
    (void)hipFree(c->d_ctiles);
    (void)hipFree(c->d_ftiles);
    (void)hipFree(c->d_step);
    (void)hipFree(c->d_fault);
    (void)hipFree(c->d_rows);
    (void)hipFree(c->d_inv);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
}

// ---------------------------------------------------------------- kernels --
using Fn3 = void (*)(StepArgs3);

template <class S, class T, int FLOW, bool WALLS, bool FIELDS>
Fn3 pick_shape3(int ty, bool nt) {
    if constexpr (FIELDS) {
        return k_collide3<S, T, FLOW, WALLS, FTY, true, false>;
    } else {
        if (ty == 8)
            return nt ? k_collide3<S, T, FLOW, WALLS, 8, false, true>
                      : k_collide3<S, T, FLOW, WALLS, 8, false, false>;
        return nt ? k_collide3<S, T, FLOW, WALLS, 4, false, true>
                  : k_collide3<S, T, FLOW, WALLS, 4, false, false>;
    }
}
template <class S, class T, bool FIELDS>
Fn3 pick_collide_t(int flow, int walls, int ty, bool nt) {
    if (flow == FLOW_NONE)
        return walls ? pick_shape3<S, T, FLOW_NONE, true, FIELDS>(ty, nt)
                     : pick_shape3<S, T, FLOW_NONE, false, FIELDS>(ty, nt);
    if (flow == FLOW_PRESCRIBED)
        return walls ? pick_shape3<S, T, FLOW_PRESCRIBED, true, FIELDS>(ty, nt)
                     : pick_shape3<S, T, FLOW_PRESCRIBED, false, FIELDS>(ty, nt);
    return walls ? pick_shape3<S, T, FLOW_COUPLED, true, FIELDS>(ty, nt)
                 : pick_shape3<S, T, FLOW_COUPLED, false, FIELDS>(ty, nt);
}
template <class S, class T>
Fn3 pick_moments_t(int flow, int walls) {
    if (flow == FLOW_COUPLED)
        return walls ? k_moments3<S, T, FLOW_COUPLED, true> : k_moments3<S, T, FLOW_COUPLED, false>;
    return walls ? k_moments3<S, T, FLOW_NONE, true> : k_moments3<S, T, FLOW_NONE, false>;
}
// non-temporal population stores when the two population buffers exceed the
// last-level cache (256 MiB Infinity Cache on MI355X): the write stream then
// does not evict lines that neighbouring columns still read
constexpr int64_t LLC_BYTES3 = int64_t(256) << 20;
bool stores_nt3(const cmlb3_ctx* c) {
    if (c->store_policy == 1) return false;
    if (c->store_policy == 2) return true;
    return 2 * c->pop_bytes > LLC_BYTES3;
}

Fn3 pick_collide(const cmlb3_ctx* c, bool fields) {
    const int ty = c->cty;
    const bool nt = stores_nt3(c);
    if (c->prec == CMLB_FP64)
        return fields ? pick_collide_t<double, double, true>(c->flow, c->walls, ty, nt)
                      : pick_collide_t<double, double, false>(c->flow, c->walls, ty, nt);
    if (c->prec == CMLB_FP32)
        return fields ? pick_collide_t<float, float, true>(c->flow, c->walls, ty, nt)
                      : pick_collide_t<float, float, false>(c->flow, c->walls, ty, nt);
    return fields ? pick_collide_t<_Float16, float, true>(c->flow, c->walls, ty, nt)
                  : pick_collide_t<_Float16, float, false>(c->flow, c->walls, ty, nt);
}
Fn3 pick_moments(const cmlb3_ctx* c) {
    if (c->prec == CMLB_FP64) return pick_moments_t<double, double>(c->flow, c->walls);
    if (c->prec == CMLB_FP32) return pick_moments_t<float, float>(c->flow, c->walls);
    return pick_moments_t<_Float16, float>(c->flow, c->walls);
}

int grid_of(int ntiles) { return (ntiles + 7) / 8 * 8; }

StepArgs3 args3(cmlb3_ctx* c, int parity, bool moments) {
    StepArgs3 a;
    memset(&a, 0, sizeof(a));
    a.src = c->pop[parity];
    a.dst = c->pop[parity ^ 1];
    a.mom = c->mom;
    a.sims = c->d_sims;
    a.tiles = moments ? c->d_mtiles : c->d_ctiles;
    a.tile_base = 0;
    a.ntiles = moments ? c->n_mtiles : c->n_ctiles;
    a.xcd_remap = 1;
    a.zseg = c->czs;
    a.ushape = c->ushape;
    a.step_in = c->d_step + parity;
    a.step_out = c->d_step + (parity ^ 1);
    a.fault = c->d_fault;
    return a;
}

int launch_pair(cmlb3_ctx* c, int parity) {
    StepArgs3 am = args3(c, parity, true);
    hipLaunchKernelGGL(pick_moments(c), dim3(grid_of(c->n_mtiles)), dim3(WG3), 0, c->stream, am);
    HIP3(c, hipGetLastError());
    StepArgs3 ac = args3(c, parity, false);
    hipLaunchKernelGGL(pick_collide(c, false), dim3(grid_of(c->n_ctiles)), dim3(c->cty * 64), 0,
                       c->stream, ac);
    HIP3(c, hipGetLastError());
    return CMLB_OK;
}

int build_graph3(cmlb3_ctx* c, int p) {
    HIP3(c, hipGraphCreate(&c->graph[p], 0));
    hipGraphNode_t prev = nullptr;
    for (int s = 0; s < GRAPH_STEPS3; ++s) {
        for (int half = 0; half < 2; ++half) {
            const bool mom = half == 0;
            StepArgs3 a = args3(c, p ^ (s & 1), mom);
            void* kargs[] = {&a};
            hipKernelNodeParams np;
            memset(&np, 0, sizeof(np));
            np.func = reinterpret_cast<void*>(mom ? pick_moments(c) : pick_collide(c, false));
            np.gridDim = dim3(grid_of(mom ? c->n_mtiles : c->n_ctiles));
            np.blockDim = dim3(mom ? WG3 : c->cty * 64);
            np.kernelParams = kargs;
            hipGraphNode_t node;
            HIP3(c, hipGraphAddKernelNode(&node, c->graph[p], prev ? &prev : nullptr, prev ? 1 : 0,
                                          &np));
            prev = node;
        }
    }
    HIP3(c, hipGraphInstantiate(&c->gexec[p], c->graph[p], nullptr, nullptr, 0));
    return CMLB_OK;
}

// collision columns (64 x ty nodes, zs planes from z0) of every simulation
// (z-major, then y, then x)
std::vector<int4> collide_tiles(const std::vector<cmlb3_sim_params>& ps, int ty, int zs,
                                std::vector<int>* first, std::vector<int>* count) {
    std::vector<int4> ct;
    for (int s = 0; s < (int)ps.size(); ++s) {
        const cmlb3_sim_params& p = ps[s];
        if (first) first->push_back((int)ct.size());
        for (int z0 = 0; z0 < p.nz; z0 += zs)
            for (int y0 = 0; y0 < p.ny; y0 += ty)
                for (int x0 = 0; x0 < p.nx; x0 += TXW) ct.push_back(make_int4(s, x0, y0, z0));
        if (count) count->push_back((int)ct.size() - first->back());
    }
    return ct;
}

int build_ctiles3(cmlb3_ctx* c) {
    std::vector<int4> ct = collide_tiles(c->params, c->cty, c->czs, nullptr, nullptr);
    if (c->d_ctiles) (void)hipFree(c->d_ctiles);
    c->d_ctiles = nullptr;
    c->n_ctiles = (int)ct.size();
    HIP3(c, hipMalloc(&c->d_ctiles, sizeof(int4) * ct.size()));
    HIP3(c, hipMemcpy(c->d_ctiles, ct.data(), sizeof(int4) * ct.size(), hipMemcpyHostToDevice));
    drop_graphs3(c);
    return CMLB_OK;
}

int sync_check3(cmlb3_ctx* c) {
    HIP3(c, hipStreamSynchronize(c->stream));
    std::vector<int32_t> f(c->n_sims);
    HIP3(c, hipMemcpy(f.data(), c->d_fault, sizeof(int32_t) * c->n_sims, hipMemcpyDeviceToHost));
    for (int s = 0; s < c->n_sims; ++s)
        if (f[s]) {
            c->fault_seen = true;
            return fail3(c, CMLB_ERANGE, "fault flags 0x%x raised in simulation %d", f[s], s);
        }
    return CMLB_OK;
}

bool sim_ok(const cmlb3_ctx* c, int s) { return c && s >= 0 && s < c->n_sims; }

// moments of the current state for one simulation's fields (moments launch
// over that simulation's tiles only)
int moments_of(cmlb3_ctx* c, int sim) {
    StepArgs3 am = args3(c, c->cur, true);
    const SimDev3& d = c->sims[sim];
    (void)d;
    hipLaunchKernelGGL(pick_moments(c), dim3(grid_of(c->n_mtiles)), dim3(WG3), 0, c->stream, am);
    HIP3(c, hipGetLastError());
    return CMLB_OK;
}

}  // namespace

// ==========================================================================
extern "C" {

int cmlb3_create(const cmlb3_sim_params* params, int32_t n_sims, int32_t precision,
                 void* hip_stream, cmlb3_ctx** out) {
    if (!out) return CMLB_EINVAL;
    *out = nullptr;
    if (!params || n_sims < 1) return CMLB_EINVAL;
    if (precision < CMLB_FP64 || precision > CMLB_FP16) return CMLB_EINVAL;
    const int flow = params[0].flow, bc = params[0].bc_y;
    if (flow < CMLB_FLOW_NONE || flow > CMLB_FLOW_COUPLED) return CMLB_EINVAL;
    if (bc != CMLB_BC_PERIODIC && bc != CMLB_BC_MOVING_WALLS) return CMLB_EINVAL;
    const int walls = bc == CMLB_BC_MOVING_WALLS;
    const int nlat = flow == CMLB_FLOW_COUPLED ? 3 : 2;
    const size_t sb = sbytes(precision);
    std::vector<SimDev3> sims(n_sims);
    std::vector<int4> mt;
    int64_t off = 0, moff = 0, uoff = 0, max_vol = 0, max_rows = 0, nodes = 0;
    for (int s = 0; s < n_sims; ++s) {
        const cmlb3_sim_params& p = params[s];
        if (p.flow != flow || p.bc_y != bc) return CMLB_EINVAL;
        if (p.nx < 4 || p.ny < 4 || p.nz < 1) return CMLB_EINVAL;
        const int64_t vol = (int64_t)p.nx * p.ny * p.nz;
        if (27 * vol * (int64_t)sb > (int64_t)INT32_MAX) return CMLB_EINVAL;
        if (NMOM * vol >= (int64_t)INT32_MAX) return CMLB_EINVAL;
        if (!(p.W > 0.0) || !(p.phi_a != p.phi_b) || !std::isfinite(p.phi_a) ||
            !std::isfinite(p.phi_b))
            return CMLB_EINVAL;
        if (!(p.M_phi >= 0.0) || !(p.D_s >= 0.0)) return CMLB_EINVAL;
        if (!rate_ok3(omega3(p.M_phi)) || !rate_ok3(omega3(p.D_s))) return CMLB_EUNSTABLE;
        if (flow == CMLB_FLOW_COUPLED) {
            if (!(p.rho_a > 0.0) || !(p.rho_b > 0.0) || !(p.c_max > 0.0)) return CMLB_EINVAL;
            if (!(p.nu_a >= 0.0) || !(p.nu_b >= 0.0)) return CMLB_EINVAL;
            if (!rate_ok3(omega3(p.nu_a)) || !rate_ok3(omega3(p.nu_b)) || !rate_ok3(p.omega_zeta))
                return CMLB_EUNSTABLE;
        }
        Desc3 d;
        const double phio = 0.5 * (p.phi_a - p.phi_b);
        d.P_ref = p.rho_b / 3.0;
        if (precision == CMLB_FP16) {
            d.qref_f = 0.5 * (p.phi_a + p.phi_b);
            d.scale_f = 0.5 / pow2_floor3(std::fabs(phio) * 1.0000001);
            if (!(d.scale_f > 0.0) || !std::isfinite(d.scale_f)) d.scale_f = 1.0;
            d.scale_h = 16.0 / pow2_floor3(p.c_max > 0.0 ? p.c_max : 1.0);
            // g holds 3 e_a.u P-sized velocity terms and the pressure
            // deviation, which reaches cs^2 |rho_a - rho_b| across an
            // interface when P starts at rho cs^2; values are kept near 32
            // (binary16 overflows at 65504), speeds taken as O(u_wall),
            // at least 1e-4 (as in 2D)
            const double uref = std::max(std::fabs(walls ? p.u_wall : 0.0), 1e-4);
            const double dev = std::max(3.0 * uref, std::fabs(p.rho_a - p.rho_b) / 3.0);
            d.scale_g = pow2_floor3(32.0 / dev);
        } else {
            d.qref_f = 0.0;
            d.scale_f = d.scale_h = d.scale_g = 1.0;
        }
        SimDev3 sd;
        memset(&sd, 0, sizeof(sd));
        sd.nx = p.nx;
        sd.ny = p.ny;
        sd.nz = p.nz;
        sd.uniform_rho = p.rho_a == p.rho_b;
        sd.uniform_nu = p.nu_a == p.nu_b;
        sd.off = off;
        sd.moff = moff;
        sd.uoff = uoff;
        sd.node_base = (uint32_t)nodes;
        sd.vel_period_T = p.vel_period_T;
        fill3(sd.kd, p, d, walls);
        fill3(sd.kf, p, d, walls);
        // moments tiles: 64 x MT_ROWS (y, z) rows
        const int rows = p.ny * p.nz;
        for (int r0 = 0; r0 < rows; r0 += MT_ROWS)
            for (int x0 = 0; x0 < p.nx; x0 += TXW) mt.push_back(make_int4(s, x0, r0, 0));
        sims[s] = sd;
        off += (int64_t)nlat * 27 * vol;
        moff += (int64_t)NMOM * vol;
        if (flow == CMLB_FLOW_PRESCRIBED) uoff += 3 * vol;
        nodes += vol;
        max_vol = std::max(max_vol, vol);
        max_rows = std::max<int64_t>(max_rows, (int64_t)p.ny * p.nz);
    }
    cmlb3_ctx* c = new (std::nothrow) cmlb3_ctx();
    if (!c) return CMLB_ENOMEM;
    c->n_sims = n_sims;
    c->prec = precision;
    c->flow = flow;
    c->walls = walls;
    c->nlat = nlat;
    c->params.assign(params, params + n_sims);
    c->sims = sims;
    c->inited.assign(n_sims, 0);
    c->pop_elems = off;
    c->mom_elems = moff;
    c->ushape_elems = uoff;
    c->max_vol = max_vol;
    c->max_rows = max_rows;
    c->n_mtiles = (int)mt.size();
    c->pop_bytes = (int64_t)sb * off;
    const Shape3 dsh = default_shape3(precision);
    c->cty = dsh.ty;
    c->czs = dsh.zs;
    std::vector<int4> ct = collide_tiles(c->params, c->cty, c->czs, nullptr, nullptr);
    std::vector<int4> ft = collide_tiles(c->params, FTY, FZS, &c->ftile0, &c->fntiles);
    c->n_ctiles = (int)ct.size();
    auto bail = [&](int code) {
        release3(c);
        delete c;
        return code;
    };
    if (hipGetDevice(&c->device) != hipSuccess) return bail(CMLB_EDEVICE);
    if (hip_stream) {
        c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(CMLB_EDEVICE);
        c->own_stream = true;
    }
    const size_t tb = precision == CMLB_FP64 ? 8 : 4;
    if (hipMalloc(&c->pop[0], sb * off) != hipSuccess) return bail(CMLB_ENOMEM);
    if (hipMalloc(&c->pop[1], sb * off) != hipSuccess) return bail(CMLB_ENOMEM);
    if (hipMalloc(&c->mom, tb * moff) != hipSuccess) return bail(CMLB_ENOMEM);
    if (uoff && hipMalloc(&c->ushape, tb * uoff) != hipSuccess) return bail(CMLB_ENOMEM);
    if (hipMalloc(&c->d_sims, sizeof(SimDev3) * n_sims) != hipSuccess) return bail(CMLB_ENOMEM);
    if (hipMalloc(&c->d_mtiles, sizeof(int4) * mt.size()) != hipSuccess) return bail(CMLB_ENOMEM);
    if (hipMalloc(&c->d_ctiles, sizeof(int4) * ct.size()) != hipSuccess) return bail(CMLB_ENOMEM);
    if (hipMalloc(&c->d_ftiles, sizeof(int4) * ft.size()) != hipSuccess) return bail(CMLB_ENOMEM);
    if (hipMalloc(&c->d_step, sizeof(int64_t) * 2) != hipSuccess) return bail(CMLB_ENOMEM);
    if (hipMalloc(&c->d_fault, sizeof(int32_t) * n_sims) != hipSuccess) return bail(CMLB_ENOMEM);
    if (hipMalloc(&c->d_rows, sizeof(double) * 2 * max_rows) != hipSuccess)
        return bail(CMLB_ENOMEM);
    if (hipMalloc(&c->d_inv, sizeof(double) * 2) != hipSuccess) return bail(CMLB_ENOMEM);
    if (hipMemset(c->pop[0], 0, sb * off) != hipSuccess) return bail(CMLB_EDEVICE);
    if (hipMemset(c->pop[1], 0, sb * off) != hipSuccess) return bail(CMLB_EDEVICE);
    if (hipMemset(c->mom, 0, tb * moff) != hipSuccess) return bail(CMLB_EDEVICE);
    if (hipMemset(c->d_step, 0, sizeof(int64_t) * 2) != hipSuccess) return bail(CMLB_EDEVICE);
    if (hipMemset(c->d_fault, 0, sizeof(int32_t) * n_sims) != hipSuccess) return bail(CMLB_EDEVICE);
    if (hipMemcpy(c->d_sims, sims.data(), sizeof(SimDev3) * n_sims, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(c->d_mtiles, mt.data(), sizeof(int4) * mt.size(), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(c->d_ctiles, ct.data(), sizeof(int4) * ct.size(), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(c->d_ftiles, ft.data(), sizeof(int4) * ft.size(), hipMemcpyHostToDevice) !=
            hipSuccess)
        return bail(CMLB_EDEVICE);
    *out = c;
    return CMLB_OK;
}

int cmlb3_init_fields(cmlb3_ctx* c, int32_t sim, const double* phi, const double* cc,
                      const double* ux, const double* uy, const double* uz, const double* p) {
    if (!c) return CMLB_EINVAL;
    if (!sim_ok(c, sim)) return fail3(c, CMLB_EINVAL, "bad simulation index");
    if (!phi || !cc) return fail3(c, CMLB_EINVAL, "phi and c are required");
    const SimDev3& d = c->sims[sim];
    const int64_t vol = (int64_t)d.nx * d.ny * d.nz;
    const double* host[6] = {phi, cc, ux, uy, uz, p};
    double* dev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    int rc = CMLB_OK;
    HIP3(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < 6 && rc == CMLB_OK; ++i) {
        if (!host[i]) continue;
        if (hipMalloc(&dev[i], sizeof(double) * vol) != hipSuccess) {
            rc = fail3(c, CMLB_ENOMEM, "staging allocation failed");
            break;
        }
        if (hipMemcpy(dev[i], host[i], sizeof(double) * vol, hipMemcpyHostToDevice) != hipSuccess)
            rc = fail3(c, CMLB_EDEVICE, "staging copy failed");
    }
    if (rc == CMLB_OK) {
        InitArgs3 a;
        memset(&a, 0, sizeof(a));
        const size_t sb = sbytes(c->prec), tb = c->prec == CMLB_FP64 ? 8 : 4;
        a.pop = static_cast<char*>(c->pop[c->cur]) + d.off * sb;
        a.sd = c->d_sims + sim;
        a.phi = dev[0];
        a.c = dev[1];
        a.ux = dev[2];
        a.uy = dev[3];
        a.uz = dev[4];
        a.P = dev[5];
        a.ushape = c->flow == CMLB_FLOW_PRESCRIBED ? static_cast<char*>(c->ushape) + d.uoff * tb
                                                    : nullptr;
        a.flow = c->flow;
        a.walls = c->walls;
        const int grid = (int)((vol + WG3 - 1) / WG3);
        if (c->prec == CMLB_FP64)
            hipLaunchKernelGGL((k_init3<double, double>), dim3(grid), dim3(WG3), 0, c->stream, a);
        else if (c->prec == CMLB_FP32)
            hipLaunchKernelGGL((k_init3<float, float>), dim3(grid), dim3(WG3), 0, c->stream, a);
        else
            hipLaunchKernelGGL((k_init3<_Float16, float>), dim3(grid), dim3(WG3), 0, c->stream, a);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
            rc = fail3(c, CMLB_EDEVICE, "init kernel failed");
    }
    for (int i = 0; i < 6; ++i) (void)hipFree(dev[i]);
    if (rc != CMLB_OK) return rc;
    HIP3(c, hipMemset(c->d_fault + sim, 0, sizeof(int32_t)));
    // both parities of the step counter restart at 0
    HIP3(c, hipMemset(c->d_step, 0, sizeof(int64_t) * 2));
    c->step = 0;
    c->fault_seen = false;
    c->inited[sim] = 1;
    return CMLB_OK;
}

int cmlb3_step(cmlb3_ctx* c, int32_t n) {
    if (!c) return CMLB_EINVAL;
    if (n < 0) return fail3(c, CMLB_EINVAL, "negative step count");
    for (int s = 0; s < c->n_sims; ++s)
        if (!c->inited[s]) return fail3(c, CMLB_ESTATE, "simulation %d not initialised", s);
    if (c->fault_seen) return fail3(c, CMLB_ERANGE, "a fault flag was raised earlier");
    int left = n;
    if (c->use_graph) {
        while (left >= GRAPH_STEPS3) {
            const int p = c->cur;
            if (!c->gexec[p]) {
                int rc = build_graph3(c, p);
                if (rc != CMLB_OK) return rc;
            }
            HIP3(c, hipGraphLaunch(c->gexec[p], c->stream));
            left -= GRAPH_STEPS3;
            c->step += GRAPH_STEPS3;
        }
    }
    while (left > 0) {
        int rc = launch_pair(c, c->cur);
        if (rc != CMLB_OK) return rc;
        c->cur ^= 1;
        c->step += 1;
        --left;
    }
    return CMLB_OK;
}

int cmlb3_read_fields(cmlb3_ctx* c, int32_t sim, double* phi, double* cc, double* ux,
                      double* uy, double* uz, double* p) {
    if (!c) return CMLB_EINVAL;
    if (!sim_ok(c, sim)) return fail3(c, CMLB_EINVAL, "bad simulation index");
    const SimDev3& d = c->sims[sim];
    const int64_t vol = (int64_t)d.nx * d.ny * d.nz;
    double* stage = nullptr;
    if (hipMalloc(&stage, sizeof(double) * 6 * vol) != hipSuccess)
        return fail3(c, CMLB_ENOMEM, "staging allocation failed");
    int rc = moments_of(c, sim);
    if (rc == CMLB_OK) {
        StepArgs3 a = args3(c, c->cur, false);
        a.dst = nullptr;
        a.step_out = nullptr;
        a.tiles = c->d_ftiles;
        a.tile_base = c->ftile0[sim];
        a.ntiles = c->fntiles[sim];
        a.xcd_remap = 0;
        a.zseg = FZS;
        a.fields_out = stage;
        hipLaunchKernelGGL(pick_collide(c, true), dim3(c->fntiles[sim]), dim3(FTY * 64), 0,
                           c->stream, a);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
            rc = fail3(c, CMLB_EDEVICE, "field kernel failed");
    }
    double* outs[6] = {phi, cc, ux, uy, uz, p};
    for (int f = 0; f < 6 && rc == CMLB_OK; ++f)
        if (outs[f] && hipMemcpy(outs[f], stage + f * vol, sizeof(double) * vol,
                                 hipMemcpyDeviceToHost) != hipSuccess)
            rc = fail3(c, CMLB_EDEVICE, "field copy failed");
    (void)hipFree(stage);
    if (rc != CMLB_OK) return rc;
    return sync_check3(c);
}

int cmlb3_inventory(cmlb3_ctx* c, int32_t sim, double* sum_phi, double* sum_c) {
    if (!c) return CMLB_EINVAL;
    if (!sim_ok(c, sim)) return fail3(c, CMLB_EINVAL, "bad simulation index");
    const SimDev3& d = c->sims[sim];
    const int rows = d.ny * d.nz;
    const size_t sb = sbytes(c->prec);
    const void* pop = static_cast<const char*>(c->pop[c->cur]) + d.off * sb;
    if (c->prec == CMLB_FP64)
        hipLaunchKernelGGL(k_inventory_rows3<double>, dim3(rows, 2), dim3(WG3), 0, c->stream, pop,
                           c->d_sims + sim, c->d_rows);
    else if (c->prec == CMLB_FP32)
        hipLaunchKernelGGL(k_inventory_rows3<float>, dim3(rows, 2), dim3(WG3), 0, c->stream, pop,
                           c->d_sims + sim, c->d_rows);
    else
        hipLaunchKernelGGL(k_inventory_rows3<_Float16>, dim3(rows, 2), dim3(WG3), 0, c->stream,
                           pop, c->d_sims + sim, c->d_rows);
    HIP3(c, hipGetLastError());
    hipLaunchKernelGGL(k_inventory_final3, dim3(1), dim3(WG3), 0, c->stream, c->d_rows, rows,
                       c->d_inv);
    HIP3(c, hipGetLastError());
    double out[2];
    HIP3(c, hipStreamSynchronize(c->stream));
    HIP3(c, hipMemcpy(out, c->d_inv, sizeof(out), hipMemcpyDeviceToHost));
    if (sum_phi) *sum_phi = out[0];
    if (sum_c) *sum_c = out[1];
    return CMLB_OK;
}

static int transfer3(cmlb3_ctx* c, int32_t sim, double* f, double* h, double* g, int dir) {
    if (!c) return CMLB_EINVAL;
    if (!sim_ok(c, sim)) return fail3(c, CMLB_EINVAL, "bad simulation index");
    const SimDev3& d = c->sims[sim];
    const int64_t vol = (int64_t)d.nx * d.ny * d.nz;
    const int nl = c->nlat;
    double* stage = nullptr;
    if (hipMalloc(&stage, sizeof(double) * nl * 27 * vol) != hipSuccess)
        return fail3(c, CMLB_ENOMEM, "staging allocation failed");
    double* host[3] = {f, h, g};
    int rc = CMLB_OK;
    HIP3(c, hipStreamSynchronize(c->stream));
    if (dir == 1)
        for (int l = 0; l < nl && rc == CMLB_OK; ++l)
            if (hipMemcpy(stage + l * 27 * vol, host[l], sizeof(double) * 27 * vol,
                          hipMemcpyHostToDevice) != hipSuccess)
                rc = fail3(c, CMLB_EDEVICE, "population copy failed");
    if (rc == CMLB_OK) {
        const size_t sb = sbytes(c->prec);
        void* pop = static_cast<char*>(c->pop[c->cur]) + d.off * sb;
        const int grid = (int)((nl * 27 * vol + WG3 - 1) / WG3);
        if (c->prec == CMLB_FP64)
            hipLaunchKernelGGL((k_transfer3<double, double>), dim3(grid), dim3(WG3), 0, c->stream,
                               pop, c->d_sims + sim, stage, nl, c->walls, dir);
        else if (c->prec == CMLB_FP32)
            hipLaunchKernelGGL((k_transfer3<float, float>), dim3(grid), dim3(WG3), 0, c->stream,
                               pop, c->d_sims + sim, stage, nl, c->walls, dir);
        else
            hipLaunchKernelGGL((k_transfer3<_Float16, float>), dim3(grid), dim3(WG3), 0,
                               c->stream, pop, c->d_sims + sim, stage, nl, c->walls, dir);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
            rc = fail3(c, CMLB_EDEVICE, "population transfer kernel failed");
    }
    if (dir == 0)
        for (int l = 0; l < nl && rc == CMLB_OK; ++l)
            if (host[l] && hipMemcpy(host[l], stage + l * 27 * vol, sizeof(double) * 27 * vol,
                                     hipMemcpyDeviceToHost) != hipSuccess)
                rc = fail3(c, CMLB_EDEVICE, "population copy failed");
    (void)hipFree(stage);
    return rc;
}

int cmlb3_get_populations(cmlb3_ctx* c, int32_t sim, double* f, double* h, double* g) {
    if (c && c->flow != CMLB_FLOW_COUPLED) g = nullptr;
    return transfer3(c, sim, f, h, g, 0);
}

int cmlb3_set_populations(cmlb3_ctx* c, int32_t sim, const double* f, const double* h,
                          const double* g) {
    if (!c) return CMLB_EINVAL;
    if (!f || !h || (c->flow == CMLB_FLOW_COUPLED && !g))
        return fail3(c, CMLB_EINVAL, "f and h (and g when coupled) are required");
    return transfer3(c, sim, const_cast<double*>(f), const_cast<double*>(h),
                     const_cast<double*>(g), 1);
}

int cmlb3_fault_flags(cmlb3_ctx* c, int32_t sim, int32_t* flags) {
    if (!c || !flags) return CMLB_EINVAL;
    if (!sim_ok(c, sim)) return fail3(c, CMLB_EINVAL, "bad simulation index");
    HIP3(c, hipStreamSynchronize(c->stream));
    HIP3(c, hipMemcpy(flags, c->d_fault + sim, sizeof(int32_t), hipMemcpyDeviceToHost));
    return CMLB_OK;
}

int cmlb3_synchronize(cmlb3_ctx* c) {
    if (!c) return CMLB_EINVAL;
    return sync_check3(c);
}

int cmlb3_set_tile_shape(cmlb3_ctx* c, int32_t ty, int32_t zs) {
    if (!c) return CMLB_EINVAL;
    if (ty == 0 && zs == 0) {
        const Shape3 d = default_shape3(c->prec);
        ty = d.ty;
        zs = d.zs;
    }
    bool ok = false;
    for (int i = 0; i < N_SHAPES3; ++i) ok |= SHAPES3[i].ty == ty && SHAPES3[i].zs == zs;
    if (!ok) return fail3(c, CMLB_EINVAL, "collision column 64x%d over %d planes not supported", ty, zs);
    HIP3(c, hipStreamSynchronize(c->stream));
    c->cty = ty;
    c->czs = zs;
    return build_ctiles3(c);
}

int cmlb3_launch_options(const cmlb3_ctx* c, int32_t* shapes, int32_t cap) {
    if (!c || (!shapes && cap > 0)) return CMLB_EINVAL;
    for (int i = 0; i < N_SHAPES3 && 2 * i + 1 < cap; ++i) {
        shapes[2 * i] = SHAPES3[i].ty;
        shapes[2 * i + 1] = SHAPES3[i].zs;
    }
    return N_SHAPES3;
}

int cmlb3_set_store_policy(cmlb3_ctx* c, int32_t policy) {
    if (!c || policy < 0 || policy > 2) return CMLB_EINVAL;
    HIP3(c, hipStreamSynchronize(c->stream));
    c->store_policy = policy;
    drop_graphs3(c);
    return CMLB_OK;
}

int cmlb3_autotune(cmlb3_ctx* c, int32_t steps, int32_t* ty, int32_t* zs, int32_t* policy) {
    if (!c || steps < 1 || steps > 100000) return CMLB_EINVAL;
    for (int s = 0; s < c->n_sims; ++s)
        if (!c->inited[s]) return fail3(c, CMLB_ESTATE, "simulation %d not initialised", s);
    if (c->fault_seen) return fail3(c, CMLB_ERANGE, "a fault flag was raised earlier");
    HIP3(c, hipStreamSynchronize(c->stream));
    const int cur0 = c->cur;
    const int64_t step0 = c->step;
    const int ty0 = c->cty, zs0 = c->czs, p0 = c->store_policy;
    int64_t dstep[2];
    std::vector<int32_t> fault(c->n_sims);
    HIP3(c, hipMemcpy(dstep, c->d_step, sizeof(dstep), hipMemcpyDeviceToHost));
    HIP3(c, hipMemcpy(fault.data(), c->d_fault, sizeof(int32_t) * c->n_sims,
                      hipMemcpyDeviceToHost));
    void* save = nullptr;
    if (hipMalloc(&save, c->pop_bytes) != hipSuccess)
        return fail3(c, CMLB_ENOMEM, "no device memory for the autotuner's state copy");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = CMLB_OK;
    // the moment arrays are recomputed from the populations every step, so
    // the populations, the step counter and the fault flags are the state
    auto restore = [&]() -> int {
        c->cur = cur0;
        c->step = step0;
        HIP3(c, hipMemcpyAsync(c->pop[cur0], save, c->pop_bytes, hipMemcpyDeviceToDevice,
                               c->stream));
        HIP3(c, hipMemcpyAsync(c->d_step, dstep, sizeof(dstep), hipMemcpyHostToDevice,
                               c->stream));
        HIP3(c, hipMemcpyAsync(c->d_fault, fault.data(), sizeof(int32_t) * c->n_sims,
                               hipMemcpyHostToDevice, c->stream));
        HIP3(c, hipStreamSynchronize(c->stream));
        return CMLB_OK;
    };
    float best = 0.f;
    int bty = 0, bzs = 0, bp = 0;
    do {
        if (hipMemcpyAsync(save, c->pop[cur0], c->pop_bytes, hipMemcpyDeviceToDevice,
                           c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess ||
            hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            rc = fail3(c, CMLB_EDEVICE, "autotuner set-up failed");
            break;
        }
        for (int i = 0; i < N_SHAPES3 && rc == CMLB_OK; ++i)
            for (int pol = 1; pol <= 2 && rc == CMLB_OK; ++pol) {
                c->cty = SHAPES3[i].ty;
                c->czs = SHAPES3[i].zs;
                c->store_policy = pol;
                if ((rc = build_ctiles3(c)) != CMLB_OK) break;
                // untimed: builds the graph the timed steps replay
                if ((rc = cmlb3_step(c, GRAPH_STEPS3 + 2)) != CMLB_OK) break;
                if (hipEventRecord(e0, c->stream) != hipSuccess) { rc = CMLB_EDEVICE; break; }
                if ((rc = cmlb3_step(c, steps)) != CMLB_OK) break;
                float ms = 0.f;
                if (hipEventRecord(e1, c->stream) != hipSuccess ||
                    hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    rc = fail3(c, CMLB_EDEVICE, "autotuner timing failed");
                    break;
                }
                if (bty == 0 || ms < best) {
                    best = ms;
                    bty = SHAPES3[i].ty;
                    bzs = SHAPES3[i].zs;
                    bp = pol;
                }
                if ((rc = restore()) != CMLB_OK) break;
            }
    } while (false);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc != CMLB_OK) {
        (void)restore();
        (void)hipFree(save);
        c->cty = ty0;
        c->czs = zs0;
        c->store_policy = p0;
        (void)build_ctiles3(c);
        return rc;
    }
    (void)hipFree(save);
    c->cty = bty;
    c->czs = bzs;
    c->store_policy = bp;
    if ((rc = build_ctiles3(c)) != CMLB_OK) return rc;
    if (ty) *ty = bty;
    if (zs) *zs = bzs;
    if (policy) *policy = bp;
    return CMLB_OK;
}

int cmlb3_set_use_graph(cmlb3_ctx* c, int32_t on) {
    if (!c) return CMLB_EINVAL;
    c->use_graph = on ? 1 : 0;
    return CMLB_OK;
}

int64_t cmlb3_step_count(const cmlb3_ctx* c) { return c ? c->step : -1; }
const char* cmlb3_last_error(const cmlb3_ctx* c) { return c ? c->err.c_str() : "null context"; }

void cmlb3_destroy(cmlb3_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    release3(c);
    delete c;
}

}  // extern "C"
