// Host runtime and C ABI (include/cmlb.h) of the MI355X coupled
// central-moment LB step.  Owns device buffers, the tile tables, the step
// counter and the HIP graphs; every step runs in the kernels of kernels.hpp.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cmlb.h"
#include "kernels.hpp"

using namespace cmlb;

namespace cmlb {
typedef float f32x4 __attribute__((ext_vector_type(4)));
// Plain device copy (cmlb_copy): four 16-byte loads per thread, then four
// stores; NT marks both non-temporal.
template <bool NT>
__global__ __launch_bounds__(256) void k_copy(const f32x4* __restrict__ a, f32x4* __restrict__ b,
                                              int64_t n4) {
    const int64_t base = (int64_t)blockIdx.x * (4 * 256) + threadIdx.x;
    f32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = base + (int64_t)u * 256;
        if (i < n4) v[u] = NT ? __builtin_nontemporal_load(&a[i]) : a[i];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = base + (int64_t)u * 256;
        if (i < n4) {
            if (NT) __builtin_nontemporal_store(v[u], &b[i]);
            else b[i] = v[u];
        }
    }
}
// Structure-of-arrays copy (cmlb_copy_planes): P planes of n4 vectors; each
// thread loads one 16-byte vector of every plane, then stores them, so P read
// and P write streams are open at once, as in a step over P direction planes.
template <int P, bool NT>
__global__ __launch_bounds__(256) void k_copy_planes(const f32x4* __restrict__ a,
                                                     f32x4* __restrict__ b, int64_t n4) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n4) return;
    f32x4 v[P];
#pragma unroll
    for (int q = 0; q < P; ++q) v[q] = NT ? __builtin_nontemporal_load(&a[q * n4 + i]) : a[q * n4 + i];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        if (NT) __builtin_nontemporal_store(v[q], &b[q * n4 + i]);
        else b[q * n4 + i] = v[q];
    }
}
// Launch-cost probes (cmlb_launch_costs): a loop of grid barriers in one
// cooperative launch, and a kernel that does nothing (its store is never
// taken: no thread index reaches 2^20).
__global__ __launch_bounds__(256) void k_grid_sync_loop(int32_t iters, float* sink) {
    cooperative_groups::grid_group g = cooperative_groups::this_grid();
    float acc = float(threadIdx.x);
    for (int i = 0; i < iters; ++i) {
        acc = acc * 0.5f + 1.0f;
        g.sync();
    }
    if (threadIdx.x >= (1u << 20)) sink[blockIdx.x] = acc;
}
__global__ __launch_bounds__(256) void k_nothing(float* sink) {
    if (threadIdx.x >= (1u << 20)) sink[blockIdx.x] = 1.0f;
}
}  // namespace cmlb

namespace {

// Scratch of the allocation-free inventory entry point
// (cmlb_inventories_noalloc): the row partials live in this file-scope
// device array, one copy per GPU, held until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in): the device address is looked up once per device with
// hipGetSymbolAddress at context creation and used from then on.
constexpr int SCRATCH_ROWS = CMLB_NOALLOC_MAX_ROWS;
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
hipError_t g_scratch_err[MAX_DEVICES] = {};

}  // namespace

static __device__ __align__(256) double scratch[2 * SCRATCH_ROWS];

namespace {

// Device address of `scratch` on the current device `device` (looked up
// once per device; nullptr if the lookup failed, the error in *err).
void* scratch_on(int device, hipError_t* err) {
    *err = hipErrorInvalidDevice;
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device] && g_scratch_err[device] == hipSuccess) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e == hipSuccess && p)
            g_scratch_ptr[device] = p;
        else
            g_scratch_err[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
    }
    *err = g_scratch_err[device];
    return g_scratch_ptr[device];
}

constexpr int GRAPH_PAIRS = 8;  // a graph holds 2 * GRAPH_PAIRS steps

size_t storage_bytes(int prec) { return prec == CMLB_FP64 ? 8 : (prec == CMLB_FP32 ? 4 : 2); }

double omega_of(double coeff) { return 1.0 / (coeff * 3.0 + 0.5); }

bool rate_ok(double w) { return std::isfinite(w) && w > 0.0 && w < 2.0; }

double pow2_floor(double v) { return std::ldexp(1.0, (int)std::floor(std::log2(v))); }

// Constants of one simulation in the compute type T.
template <class T>
void fill_consts(PhysConsts<T>& k, const SimDev& d) {
    k.inv_f = T(1.0 / d.scale_f);
    k.qref_f = T(d.qref_f);
    k.inv_h = T(1.0 / d.scale_h);
    k.inv_g = T(1.0 / d.scale_g);
    // the weight rounded to T first, then scaled by the power of two 1/scale_g
    // (exact): v * wdec equals w_a * (v / scale_g) bit for bit
    k.wdec0 = T(T(4.0 / 9.0) * T(1.0 / d.scale_g));
    k.wdec1 = T(T(1.0 / 9.0) * T(1.0 / d.scale_g));
    k.wdec5 = T(T(1.0 / 36.0) * T(1.0 / d.scale_g));
    k.scale_f = T(d.scale_f);
    k.scale_h = T(d.scale_h);
    k.scale_g = T(d.scale_g);
    k.phi_a = T(d.phi_a);
    k.phi_b = T(d.phi_b);
    k.inv_dphi = T(d.inv_dphi);
    k.phim = T(d.phim);
    k.theta_k = T(d.theta_k);
    k.thetac_k = T(d.thetac_k);
    k.M_phi = T(d.M_phi);
    k.D_s = T(d.D_s);
    k.omega_k = T(d.omega_k);
    k.omega_c = T(d.omega_c);
    k.rho_b = T(d.rho_b);
    k.drho = T(d.drho);
    k.nu_b = T(d.nu_b);
    k.dnu = T(d.dnu);
    k.inv_rho_b = T(1.0 / d.rho_b);
    k.omega_nu_b = T(1.0 / (3.0 * d.nu_b + 0.5));
    k.omega_zeta = T(d.omega_zeta);
    k.sigma0 = T(d.sigma0);
    k.beta = T(d.beta);
    k.c_max = T(d.c_max);
    k.inv_cmax = T(d.c_max != 0.0 ? 1.0 / d.c_max : 0.0);
    k.ks = T(d.ks);
    k.u_wall = T(d.u_wall);
    k.Fx = T(d.F_ext_x);
    k.Fy = T(d.F_ext_y);
    k.P_ref = T(d.P_ref);
    k.dr_cs2 = T(d.drho * d.inv_dphi / 3.0);
}

}  // namespace

struct cmlb_ctx {
    int n_sims = 0;
    int prec = 0;
    int flow = 0;
    int walls = 0;
    int nlat = 2;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    std::vector<cmlb_sim_params> params;
    std::vector<SimDev> sims;
    std::vector<char> inited;
    int64_t pop_elems = 0;
    int64_t ushape_elems = 0;
    int64_t max_plane = 0;
    int max_ny = 0;
    void* pop[2] = {nullptr, nullptr};
    void* ushape = nullptr;
    SimDev* d_sims = nullptr;
    int4* d_tiles = nullptr;
    int ntiles = 0;
    int4* d_ftiles = nullptr;        // field-evaluation tiles (64 x 8)
    std::vector<int> ftile0, fntiles;
    int64_t* d_step = nullptr;  // [2]
    int32_t* d_fault = nullptr; // [n_sims]
    double* d_stage = nullptr;  // staging: max(27, 5) * max_plane doubles
    double* d_rows = nullptr;   // inventory row partials: 2 per row of every sim
    double* d_inv = nullptr;    // inventory totals: 2 per sim
    void* scratch = nullptr;    // this device's scratch array (allocation-free entry point)
    hipError_t scratch_err = hipSuccess;
    int cur = 0;                // population/counter parity holding the current state
    int64_t step = 0;
    int tile_rows = 0;          // 0 = default
    int tile_w = 0;             // 0 = default
    int use_graph = 1;
    int xcd_remap = 1;
    int tile_group = 0;         // column-group width of the tile order (0: row-major)
    int store_policy = 0;       // 0 auto, 1 default stores, 2 non-temporal stores
    size_t pop_bytes = 0;       // bytes of one population buffer
    bool fault_seen = false;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    std::string err;
};

namespace {

int fail(cmlb_ctx* c, int code, const char* fmt, ...) {
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

#define HIP_TRY(ctx, expr)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((ctx), CMLB_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Launch shapes of the step kernel: tile = width x rows, width = 64 per
// wavefront across x, rows = (waves / wavefronts across) * rows per thread.
// FP64 keeps 4-wave workgroups (its registers allow two waves per SIMD); the
// FP32-arithmetic forms also offer 8- and 16-wave workgroups at two rows per
// thread (four waves per SIMD).  128-column tiles fetch fewer partly-used
// cache lines at their x edges.
struct Shape {
    int width, rows, nw, npt, wx;  // tile = width x rows; nw waves, wx of them across x
};
const Shape SHAPES_64[] = {{64, 4, 4, 1, 1}, {64, 8, 4, 2, 1}, {128, 4, 4, 2, 2}};
const Shape SHAPES_32[] = {{64, 4, 4, 1, 1},   {64, 8, 4, 2, 1},   {64, 16, 8, 2, 1},
                           {64, 32, 16, 2, 1}, {128, 8, 8, 2, 2},  {128, 16, 16, 2, 2}};
constexpr int N_SHAPES_64 = sizeof(SHAPES_64) / sizeof(Shape);
constexpr int N_SHAPES_32 = sizeof(SHAPES_32) / sizeof(Shape);

// the field-evaluation kernel's fixed launch: 64 x 8 tiles of 4 waves
constexpr int FIELD_NW = 4, FIELD_NPT = 2, FIELD_ROWS = FIELD_NW * FIELD_NPT;

// defaults measured on the 64-drop batch: FP64 64x8 (4 waves), FP32/FP16
// 128x8 (8 waves, two across x)
int default_width(int prec) { return prec == CMLB_FP64 ? 64 : 128; }
int default_rows(int) { return 8; }

bool shape_of(int prec, int width, int rows, Shape* out) {
    const Shape* t = prec == CMLB_FP64 ? SHAPES_64 : SHAPES_32;
    const int n = prec == CMLB_FP64 ? N_SHAPES_64 : N_SHAPES_32;
    for (int i = 0; i < n; ++i)
        if (t[i].width == width && t[i].rows == rows) {
            if (out) *out = t[i];
            return true;
        }
    return false;
}

// ------------------------------------------------------------------------
// kernel selection
// ------------------------------------------------------------------------
using StepFn = void (*)(StepArgs);

template <class S, class T, int FLOW, bool WALLS, bool FIELDS, bool NTS>
StepFn pick_shape(const Shape& sh) {
    if constexpr (FIELDS) {
        return k_step<S, T, FLOW, WALLS, FIELD_NW, FIELD_NPT, true, false, 1>;
    } else {
        if (sh.wx == 1) {
            if (sh.nw == 4 && sh.npt == 1) return k_step<S, T, FLOW, WALLS, 4, 1, false, NTS, 1>;
            if (sh.nw == 4 && sh.npt == 2) return k_step<S, T, FLOW, WALLS, 4, 2, false, NTS, 1>;
            if constexpr (sizeof(T) == 4) {
                if (sh.nw == 8) return k_step<S, T, FLOW, WALLS, 8, 2, false, NTS, 1>;
                return k_step<S, T, FLOW, WALLS, 16, 2, false, NTS, 1>;
            }
            return k_step<S, T, FLOW, WALLS, 4, 2, false, NTS, 1>;
        }
        if constexpr (sizeof(T) == 4) {
            if (sh.nw == 8) return k_step<S, T, FLOW, WALLS, 8, 2, false, NTS, 2>;
            return k_step<S, T, FLOW, WALLS, 16, 2, false, NTS, 2>;
        }
        return k_step<S, T, FLOW, WALLS, 4, 2, false, NTS, 2>;
    }
}
template <class S, class T, int FLOW, bool WALLS, bool FIELDS>
StepFn pick_policy(const Shape& sh, bool nts) {
    if constexpr (FIELDS) return pick_shape<S, T, FLOW, WALLS, true, false>(sh);
    return nts ? pick_shape<S, T, FLOW, WALLS, false, true>(sh)
               : pick_shape<S, T, FLOW, WALLS, false, false>(sh);
}
template <class S, class T, bool FIELDS>
StepFn pick_flow(int flow, int walls, const Shape& sh, bool nts) {
    if (flow == FLOW_NONE)
        return walls ? pick_policy<S, T, FLOW_NONE, true, FIELDS>(sh, nts)
                     : pick_policy<S, T, FLOW_NONE, false, FIELDS>(sh, nts);
    if (flow == FLOW_PRESCRIBED)
        return walls ? pick_policy<S, T, FLOW_PRESCRIBED, true, FIELDS>(sh, nts)
                     : pick_policy<S, T, FLOW_PRESCRIBED, false, FIELDS>(sh, nts);
    return walls ? pick_policy<S, T, FLOW_COUPLED, true, FIELDS>(sh, nts)
                 : pick_policy<S, T, FLOW_COUPLED, false, FIELDS>(sh, nts);
}
StepFn pick_step(int prec, int flow, int walls, const Shape& sh, bool fields, bool nts) {
    if (prec == CMLB_FP64)
        return fields ? pick_flow<double, double, true>(flow, walls, sh, false)
                      : pick_flow<double, double, false>(flow, walls, sh, nts);
    if (prec == CMLB_FP32)
        return fields ? pick_flow<float, float, true>(flow, walls, sh, false)
                      : pick_flow<float, float, false>(flow, walls, sh, nts);
    return fields ? pick_flow<_Float16, float, true>(flow, walls, sh, false)
                  : pick_flow<_Float16, float, false>(flow, walls, sh, nts);
}

// Population stores bypass-allocate (non-temporal) when the two population
// buffers together exceed the GPU's last-level (Infinity) cache, 256 MiB on
// MI355X: such lattices are re-read from HBM every step anyway, and streaming
// the stores keeps the L2 for the lines that neighbouring tiles share.
// Smaller lattices keep default stores, so the next step finds them cached.
constexpr size_t LLC_BYTES = size_t(256) << 20;
bool stores_nt(const cmlb_ctx* c) {
    if (c->store_policy == 1) return false;
    if (c->store_policy == 2) return true;
    return 2 * c->pop_bytes > LLC_BYTES;
}

int rows_of(const cmlb_ctx* c) { return c->tile_rows ? c->tile_rows : default_rows(c->prec); }
int width_of(const cmlb_ctx* c) { return c->tile_w ? c->tile_w : default_width(c->prec); }

void drop_graphs(cmlb_ctx* c) {
    for (int i = 0; i < 2; ++i) {
        if (c->gexec[i]) (void)hipGraphExecDestroy(c->gexec[i]);
        if (c->graph[i]) (void)hipGraphDestroy(c->graph[i]);
        c->gexec[i] = nullptr;
        c->graph[i] = nullptr;
    }
}

// Tile list.  Tiles are visited in column groups of `group` tiles (all
// rows of group 0, then group 1, ...; row-major inside a group, 0 = one
// group), so that the tiles a workgroup band has in flight at once form a
// compact patch whose rows and halos overlap in one L2.
std::vector<int4> make_tiles(const cmlb_ctx* c, int width, int rows, int group,
                             std::vector<int>* first, std::vector<int>* count) {
    std::vector<int4> tiles;
    for (int s = 0; s < c->n_sims; ++s) {
        const SimDev& d = c->sims[s];
        if (first) first->push_back((int)tiles.size());
        const int tx = (d.nx + width - 1) / width;
        const int g = group > 0 ? group : tx;
        for (int gx = 0; gx < tx; gx += g)
            for (int y0 = 0; y0 < d.ny; y0 += rows)
                for (int t = gx; t < gx + g && t < tx; ++t)
                    tiles.push_back(make_int4(s, t * width, y0, 0));
        if (count) count->push_back((int)tiles.size() - first->back());
    }
    return tiles;
}

int build_tiles(cmlb_ctx* c) {
    std::vector<int> first, count;
    std::vector<int4> tiles =
        make_tiles(c, width_of(c), rows_of(c), c->tile_group, &first, &count);
    for (int s = 0; s < c->n_sims; ++s) {
        c->sims[s].tile0 = first[s];
        c->sims[s].ntiles = count[s];
    }
    if (c->d_tiles) (void)hipFree(c->d_tiles);
    c->d_tiles = nullptr;
    c->ntiles = (int)tiles.size();
    HIP_TRY(c, hipMalloc(&c->d_tiles, sizeof(int4) * tiles.size()));
    HIP_TRY(c, hipMemcpy(c->d_tiles, tiles.data(), sizeof(int4) * tiles.size(),
                         hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_sims, c->sims.data(), sizeof(SimDev) * c->sims.size(),
                         hipMemcpyHostToDevice));
    drop_graphs(c);
    return CMLB_OK;
}

// Tiles of the field-evaluation kernel (fixed 64 x 8 shape).
int build_field_tiles(cmlb_ctx* c) {
    c->ftile0.clear();
    c->fntiles.clear();
    std::vector<int4> tiles = make_tiles(c, 64, FIELD_ROWS, 0, &c->ftile0, &c->fntiles);
    HIP_TRY(c, hipMalloc(&c->d_ftiles, sizeof(int4) * tiles.size()));
    HIP_TRY(c, hipMemcpy(c->d_ftiles, tiles.data(), sizeof(int4) * tiles.size(),
                         hipMemcpyHostToDevice));
    return CMLB_OK;
}

Shape shape_cur(const cmlb_ctx* c) {
    Shape sh{64, 8, 4, 2, 1};
    shape_of(c->prec, width_of(c), rows_of(c), &sh);
    return sh;
}

StepArgs step_args(cmlb_ctx* c, int parity) {
    StepArgs a;
    memset(&a, 0, sizeof(a));
    a.src = c->pop[parity];
    a.dst = c->pop[parity ^ 1];
    a.sims = c->d_sims;
    a.tiles = c->d_tiles;
    a.tile_base = 0;
    a.ntiles = c->ntiles;
    a.xcd_remap = c->xcd_remap;
    a.ushape = c->ushape;
    a.step_in = c->d_step + parity;
    a.step_out = c->d_step + (parity ^ 1);
    a.fault = c->d_fault;
    a.fields_out = nullptr;
    return a;
}

// grid of the step kernel: padded to a multiple of 8 when remapping per XCD
int step_grid(const cmlb_ctx* c) { return c->xcd_remap ? (c->ntiles + 7) / 8 * 8 : c->ntiles; }

int launch_step(cmlb_ctx* c, int parity) {
    const Shape sh = shape_cur(c);
    StepFn fn = pick_step(c->prec, c->flow, c->walls, sh, false, stores_nt(c));
    StepArgs a = step_args(c, parity);
    hipLaunchKernelGGL(fn, dim3(step_grid(c)), dim3(sh.nw * 64), 0, c->stream, a);
    HIP_TRY(c, hipGetLastError());
    return CMLB_OK;
}

// Graph of 2*GRAPH_PAIRS steps starting from parity p (ends at parity p).
int build_graph(cmlb_ctx* c, int p) {
    const Shape sh = shape_cur(c);
    StepFn fn = pick_step(c->prec, c->flow, c->walls, sh, false, stores_nt(c));
    HIP_TRY(c, hipGraphCreate(&c->graph[p], 0));
    hipGraphNode_t prev = nullptr;
    for (int k = 0; k < 2 * GRAPH_PAIRS; ++k) {
        StepArgs a = step_args(c, p ^ (k & 1));
        void* kargs[] = {&a};
        hipKernelNodeParams np;
        memset(&np, 0, sizeof(np));
        np.func = reinterpret_cast<void*>(fn);
        np.gridDim = dim3(step_grid(c));
        np.blockDim = dim3(sh.nw * 64);
        np.sharedMemBytes = 0;
        np.kernelParams = kargs;
        np.extra = nullptr;
        hipGraphNode_t node;
        HIP_TRY(c, hipGraphAddKernelNode(&node, c->graph[p], prev ? &prev : nullptr, prev ? 1 : 0,
                                         &np));
        prev = node;
    }
    HIP_TRY(c, hipGraphInstantiate(&c->gexec[p], c->graph[p], nullptr, nullptr, 0));
    return CMLB_OK;
}

int check_sim(const cmlb_ctx* c, int sim) { return sim >= 0 && sim < c->n_sims; }

int sync_and_check(cmlb_ctx* c) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    std::vector<int32_t> f(c->n_sims);
    HIP_TRY(c, hipMemcpy(f.data(), c->d_fault, sizeof(int32_t) * c->n_sims, hipMemcpyDeviceToHost));
    for (int s = 0; s < c->n_sims; ++s)
        if (f[s]) {
            c->fault_seen = true;
            return fail(c, CMLB_ERANGE, "fault flags 0x%x raised in simulation %d", f[s], s);
        }
    return CMLB_OK;
}

template <class S>
void launch_decode(cmlb_ctx* c, int sim) {
    const SimDev& d = c->sims[sim];
    const int64_t total = (int64_t)c->nlat * 9 * d.nx * d.ny;
    const char* base = static_cast<const char*>(c->pop[c->cur]) + d.off * (int64_t)sizeof(S);
    hipLaunchKernelGGL(k_decode<S>, dim3((unsigned)((total + WG - 1) / WG)), dim3(WG), 0,
                       c->stream, (const void*)base, (const SimDev*)(c->d_sims + sim), c->nlat,
                       c->walls, c->d_stage);
}
template <class S>
void launch_encode(cmlb_ctx* c, int sim) {
    const SimDev& d = c->sims[sim];
    const int64_t total = (int64_t)c->nlat * 9 * d.nx * d.ny;
    char* base = static_cast<char*>(c->pop[c->cur]) + d.off * (int64_t)sizeof(S);
    hipLaunchKernelGGL(k_encode<S>, dim3((unsigned)((total + WG - 1) / WG)), dim3(WG), 0,
                       c->stream, (void*)base, (const SimDev*)(c->d_sims + sim), c->nlat,
                       c->walls, (const double*)c->d_stage);
}
// Inventories of simulations [first, first + n): row partials into `rows`
// (two doubles per row of those simulations), totals into out[2 n].
template <class S>
void launch_inventory_s(cmlb_ctx* c, int first, int n, int max_ny, double* rows, double* out) {
    const int row_base = c->sims[first].row0;
    hipLaunchKernelGGL(k_inventory_rows<S>, dim3((unsigned)((int64_t)n * max_ny)), dim3(WG), 0,
                       c->stream,
                       (const void*)c->pop[c->cur], (const SimDev*)c->d_sims, c->nlat, first,
                       max_ny, row_base, rows);
    hipLaunchKernelGGL(k_inventory_final, dim3(n), dim3(WG), 0, c->stream, (const double*)rows,
                       (const SimDev*)c->d_sims, first, row_base, out);
}
int launch_inventory(cmlb_ctx* c, int first, int n, double* rows, double* out) {
    int max_ny = 0;
    for (int s = first; s < first + n; ++s) max_ny = std::max(max_ny, c->sims[s].ny);
    if ((int64_t)n * max_ny > (int64_t)INT32_MAX)
        return fail(c, CMLB_EINVAL, "too many simulation rows for one inventory launch");
    if (c->prec == CMLB_FP64)
        launch_inventory_s<double>(c, first, n, max_ny, rows, out);
    else if (c->prec == CMLB_FP32)
        launch_inventory_s<float>(c, first, n, max_ny, rows, out);
    else
        launch_inventory_s<_Float16>(c, first, n, max_ny, rows, out);
    HIP_TRY(c, hipGetLastError());
    return CMLB_OK;
}
// rows of the simulations [first, first + n)
int64_t rows_of_range(const cmlb_ctx* c, int first, int n) {
    int64_t r = 0;
    for (int s = first; s < first + n; ++s) r += c->sims[s].ny;
    return r;
}

template <class S, class T>
void launch_init(cmlb_ctx* c, int sim, const InitArgs& a) {
    const SimDev& d = c->sims[sim];
    const int plane = d.nx * d.ny;
    hipLaunchKernelGGL((k_init<S, T>), dim3((plane + WG - 1) / WG), dim3(WG), 0, c->stream, a);
}

void release(cmlb_ctx* c) {
    drop_graphs(c);
    (void)hipFree(c->pop[0]);
    (void)hipFree(c->pop[1]);
    (void)hipFree(c->ushape);
    (void)hipFree(c->d_sims);
    (void)hipFree(c->d_tiles);
    (void)hipFree(c->d_ftiles);
    (void)hipFree(c->d_step);
    (void)hipFree(c->d_fault);
    (void)hipFree(c->d_stage);
    (void)hipFree(c->d_rows);
    (void)hipFree(c->d_inv);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
}

}  // namespace

// ==========================================================================
// C ABI
// ==========================================================================
extern "C" {

int cmlb_create(const cmlb_sim_params* params, int32_t n_sims, int32_t precision,
                void* hip_stream, cmlb_ctx** out) {
    if (!out) return CMLB_EINVAL;
    *out = nullptr;
    if (!params || n_sims < 1) return CMLB_EINVAL;
    if (precision < CMLB_FP64 || precision > CMLB_FP16) return CMLB_EINVAL;
    const int flow = params[0].flow, bc = params[0].bc_y;
    if (flow < CMLB_FLOW_NONE || flow > CMLB_FLOW_COUPLED) return CMLB_EINVAL;
    if (bc != CMLB_BC_PERIODIC && bc != CMLB_BC_MOVING_WALLS) return CMLB_EINVAL;
    const int nlat = flow == CMLB_FLOW_COUPLED ? 3 : 2;
    std::vector<SimDev> sims(n_sims);
    int64_t off = 0, uoff = 0, max_plane = 0, node_count = 0, row_count = 0;
    int max_ny = 0;
    for (int s = 0; s < n_sims; ++s) {
        const cmlb_sim_params& p = params[s];
        if (p.flow != flow || p.bc_y != bc) return CMLB_EINVAL;
        if (p.nx < 4 || p.ny < 4) return CMLB_EINVAL;
        const int64_t plane = (int64_t)p.nx * p.ny;
        if (plane * 27 >= (int64_t)INT32_MAX) return CMLB_EINVAL;
        if (!(p.W > 0.0) || !(p.phi_a != p.phi_b) || !std::isfinite(p.phi_a) ||
            !std::isfinite(p.phi_b))
            return CMLB_EINVAL;
        if (!(p.M_phi >= 0.0) || !(p.D_s >= 0.0)) return CMLB_EINVAL;
        const double wk = omega_of(p.M_phi), wc = omega_of(p.D_s);
        if (!rate_ok(wk) || !rate_ok(wc)) return CMLB_EUNSTABLE;
        SimDev d;
        memset(&d, 0, sizeof(d));
        d.nx = p.nx;
        d.ny = p.ny;
        d.off = off;
        d.ushape_off = uoff;
        d.W = p.W;
        d.phi_a = p.phi_a;
        d.phi_b = p.phi_b;
        d.inv_dphi = 1.0 / (p.phi_a - p.phi_b);
        d.phim = 0.5 * (p.phi_a + p.phi_b);
        d.theta_k = 4.0 / p.W;
        d.thetac_k = 8.0 / p.W;
        d.M_phi = p.M_phi;
        d.D_s = p.D_s;
        d.omega_k = wk;
        d.omega_c = wc;
        d.rho_b = p.rho_b;
        d.drho = p.rho_a - p.rho_b;
        d.nu_b = p.nu_b;
        d.dnu = p.nu_a - p.nu_b;
        d.omega_zeta = p.omega_zeta;
        d.sigma0 = p.sigma0;
        d.beta = p.beta;
        d.c_max = p.c_max;
        const double phio = 0.5 * (p.phi_a - p.phi_b);
        d.ks = 3.0 * p.W / (8.0 * phio * phio);
        d.u_wall = bc == CMLB_BC_MOVING_WALLS ? p.u_wall : 0.0;
        d.F_ext_x = p.F_ext_x;
        d.F_ext_y = p.F_ext_y;
        d.vel_period_T = p.vel_period_T;
        d.P_ref = p.rho_b / 3.0;
        if (flow == CMLB_FLOW_COUPLED) {
            if (!(p.rho_a > 0.0) || !(p.rho_b > 0.0) || !(p.c_max > 0.0)) return CMLB_EINVAL;
            if (!(p.nu_a >= 0.0) || !(p.nu_b >= 0.0)) return CMLB_EINVAL;
            if (!rate_ok(omega_of(p.nu_a)) || !rate_ok(omega_of(p.nu_b)) || !rate_ok(p.omega_zeta))
                return CMLB_EUNSTABLE;
        }
        if (precision == CMLB_FP16) {
            // f: deviation from phi_m, bulk values map to +-1/2 exactly
            d.qref_f = d.phim;
            d.scale_f = 0.5 / pow2_floor(std::fabs(phio) * 1.0000001);
            if (!(d.scale_f > 0.0) || !std::isfinite(d.scale_f)) d.scale_f = 1.0;
            d.scale_h = 16.0 / pow2_floor(p.c_max > 0.0 ? p.c_max : 1.0);
            // g: the stored deviation q_a/w_a - P_ref holds 3 e_a.u P-sized
            // velocity terms and the pressure deviation, which reaches
            // cs^2 |rho_a - rho_b| across an interface when P starts at
            // rho cs^2; values are kept near 32 (binary16 overflows at
            // 65504).  Speeds are taken as O(u_wall), at least 1e-4.
            const double uref = std::max(std::fabs(d.u_wall), 1e-4);
            const double dev = std::max(3.0 * uref, std::fabs(p.rho_a - p.rho_b) / 3.0);
            d.scale_g = pow2_floor(32.0 / dev);
        } else {
            d.qref_f = 0.0;
            d.scale_f = d.scale_h = d.scale_g = 1.0;
        }
        // a simulation's population block (rows padded to whole runs of 64
        // nodes) must fit a 32-bit buffer range
        const int64_t nbx = (p.nx + 63) / 64;
        const int64_t row_bytes = nbx * nlat * 9 * 64 * (int64_t)storage_bytes(precision);
        if (row_bytes * p.ny > (int64_t)INT32_MAX) return CMLB_EINVAL;
        d.node_base = (uint32_t)node_count;
        if (row_count + p.ny > (int64_t)INT32_MAX) return CMLB_EINVAL;
        d.row0 = (int32_t)row_count;
        row_count += p.ny;
        d.uniform_rho = p.rho_a == p.rho_b;
        d.uniform_nu = p.nu_a == p.nu_b;
        fill_consts(d.kd, d);
        fill_consts(d.kf, d);
        sims[s] = d;
        node_count += plane;
        off += (int64_t)nlat * 9 * 64 * nbx * p.ny;  // rows padded to whole runs
        if (flow == CMLB_FLOW_PRESCRIBED) uoff += 2 * plane;
        max_plane = std::max(max_plane, plane);
        max_ny = std::max(max_ny, p.ny);
    }

    cmlb_ctx* c = new (std::nothrow) cmlb_ctx();
    if (!c) return CMLB_ENOMEM;
    c->n_sims = n_sims;
    c->prec = precision;
    c->flow = flow;
    c->walls = bc == CMLB_BC_MOVING_WALLS;
    c->nlat = nlat;
    c->params.assign(params, params + n_sims);
    c->sims = sims;
    c->inited.assign(n_sims, 0);
    c->pop_elems = off;
    c->ushape_elems = uoff;
    c->max_plane = max_plane;
    c->max_ny = max_ny;
    auto bail = [&](int code) {
        release(c);
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
    const size_t sb = storage_bytes(precision);
    const size_t tb = precision == CMLB_FP64 ? 8 : 4;
    c->pop_bytes = sb * off;
    if (hipMalloc(&c->pop[0], sb * off) != hipSuccess) return bail(CMLB_ENOMEM);
    if (hipMalloc(&c->pop[1], sb * off) != hipSuccess) return bail(CMLB_ENOMEM);
    if (uoff && hipMalloc(&c->ushape, tb * uoff) != hipSuccess) return bail(CMLB_ENOMEM);
    if (hipMalloc(&c->d_sims, sizeof(SimDev) * n_sims) != hipSuccess) return bail(CMLB_ENOMEM);
    if (hipMalloc(&c->d_step, sizeof(int64_t) * 2) != hipSuccess) return bail(CMLB_ENOMEM);
    if (hipMalloc(&c->d_fault, sizeof(int32_t) * n_sims) != hipSuccess) return bail(CMLB_ENOMEM);
    if (hipMalloc(&c->d_stage, sizeof(double) * 27 * max_plane) != hipSuccess)
        return bail(CMLB_ENOMEM);
    if (hipMalloc(&c->d_rows, sizeof(double) * 2 * row_count) != hipSuccess)
        return bail(CMLB_ENOMEM);
    if (hipMalloc(&c->d_inv, sizeof(double) * 2 * n_sims) != hipSuccess) return bail(CMLB_ENOMEM);
    c->scratch = scratch_on(c->device, &c->scratch_err);
    if (hipMemset(c->pop[0], 0, sb * off) != hipSuccess) return bail(CMLB_EDEVICE);
    if (hipMemset(c->pop[1], 0, sb * off) != hipSuccess) return bail(CMLB_EDEVICE);
    if (hipMemset(c->d_step, 0, sizeof(int64_t) * 2) != hipSuccess) return bail(CMLB_EDEVICE);
    if (hipMemset(c->d_fault, 0, sizeof(int32_t) * n_sims) != hipSuccess) return bail(CMLB_EDEVICE);
    if (build_tiles(c) != CMLB_OK) return bail(CMLB_EDEVICE);
    if (build_field_tiles(c) != CMLB_OK) return bail(CMLB_EDEVICE);
    *out = c;
    return CMLB_OK;
}

int cmlb_init_fields(cmlb_ctx* c, int32_t sim, const double* phi, const double* cc,
                     const double* ux, const double* uy, const double* p) {
    if (!c) return CMLB_EINVAL;
    if (!check_sim(c, sim) || !phi || !cc) return fail(c, CMLB_EINVAL, "bad simulation or field");
    const SimDev& d = c->sims[sim];
    const int64_t plane = (int64_t)d.nx * d.ny;
    double* st = c->d_stage;
    // staging layout: phi, c, ux, uy, P
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(st, phi, sizeof(double) * plane, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(st + plane, cc, sizeof(double) * plane, hipMemcpyHostToDevice));
    if (ux) HIP_TRY(c, hipMemcpy(st + 2 * plane, ux, sizeof(double) * plane, hipMemcpyHostToDevice));
    if (uy) HIP_TRY(c, hipMemcpy(st + 3 * plane, uy, sizeof(double) * plane, hipMemcpyHostToDevice));
    if (p) HIP_TRY(c, hipMemcpy(st + 4 * plane, p, sizeof(double) * plane, hipMemcpyHostToDevice));
    InitArgs a;
    memset(&a, 0, sizeof(a));
    a.sd = c->d_sims + sim;
    a.phi = st;
    a.c = st + plane;
    a.ux = ux ? st + 2 * plane : nullptr;
    a.uy = uy ? st + 3 * plane : nullptr;
    a.P = p ? st + 4 * plane : nullptr;
    a.flow = c->flow;
    a.walls = c->walls;
    const size_t tb = c->prec == CMLB_FP64 ? 8 : 4;
    a.ushape = c->flow == CMLB_FLOW_PRESCRIBED ? static_cast<char*>(c->ushape) + d.ushape_off * tb
                                               : nullptr;
    // initialise both copies' parity: write into the current buffer
    const size_t sb = storage_bytes(c->prec);
    a.pop = static_cast<char*>(c->pop[c->cur]) + d.off * sb;
    if (c->prec == CMLB_FP64)
        launch_init<double, double>(c, sim, a);
    else if (c->prec == CMLB_FP32)
        launch_init<float, float>(c, sim, a);
    else
        launch_init<_Float16, float>(c, sim, a);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->inited[sim] = 1;
    c->step = 0;
    int64_t zero[2] = {0, 0};
    HIP_TRY(c, hipMemcpy(c->d_step, zero, sizeof(zero), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemset(c->d_fault + sim, 0, sizeof(int32_t)));
    return CMLB_OK;
}

int cmlb_step(cmlb_ctx* c, int32_t n) {
    if (!c) return CMLB_EINVAL;
    if (n < 0) return fail(c, CMLB_EINVAL, "negative step count");
    for (int s = 0; s < c->n_sims; ++s)
        if (!c->inited[s]) return fail(c, CMLB_ESTATE, "simulation %d not initialised", s);
    if (c->fault_seen) return fail(c, CMLB_ERANGE, "a fault flag was raised earlier");
    int left = n;
    if (c->use_graph) {
        const int per = 2 * GRAPH_PAIRS;
        while (left >= per) {
            const int p = c->cur;
            if (!c->gexec[p]) {
                int rc = build_graph(c, p);
                if (rc != CMLB_OK) return rc;
            }
            HIP_TRY(c, hipGraphLaunch(c->gexec[p], c->stream));
            left -= per;
            c->step += per;
        }
    }
    while (left > 0) {
        int rc = launch_step(c, c->cur);
        if (rc != CMLB_OK) return rc;
        c->cur ^= 1;
        c->step += 1;
        --left;
    }
    return CMLB_OK;
}

int cmlb_read_fields(cmlb_ctx* c, int32_t sim, double* phi, double* cc, double* ux, double* uy,
                     double* p) {
    if (!c) return CMLB_EINVAL;
    if (!check_sim(c, sim)) return fail(c, CMLB_EINVAL, "bad simulation index");
    const SimDev& d = c->sims[sim];
    const int64_t plane = (int64_t)d.nx * d.ny;
    StepFn fn = pick_step(c->prec, c->flow, c->walls, Shape{}, true, false);
    StepArgs a = step_args(c, c->cur);
    a.dst = nullptr;
    a.step_out = nullptr;
    a.tiles = c->d_ftiles;
    a.tile_base = c->ftile0[sim];
    a.ntiles = c->fntiles[sim];
    a.xcd_remap = 0;
    a.fields_out = c->d_stage;
    hipLaunchKernelGGL(fn, dim3(c->fntiles[sim]), dim3(FIELD_NW * 64), 0, c->stream, a);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double* outs[5] = {phi, cc, ux, uy, p};
    for (int f = 0; f < 5; ++f)
        if (outs[f])
            HIP_TRY(c, hipMemcpy(outs[f], c->d_stage + f * plane, sizeof(double) * plane,
                                 hipMemcpyDeviceToHost));
    return sync_and_check(c);
}

int cmlb_inventory(cmlb_ctx* c, int32_t sim, double* sum_phi, double* sum_c) {
    if (!c) return CMLB_EINVAL;
    if (!check_sim(c, sim)) return fail(c, CMLB_EINVAL, "bad simulation index");
    int rc = launch_inventory(c, sim, 1, c->d_rows, c->d_inv);
    if (rc != CMLB_OK) return rc;
    double v[2];
    HIP_TRY(c, hipMemcpyAsync(v, c->d_inv, sizeof(v), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (sum_phi) *sum_phi = v[0];
    if (sum_c) *sum_c = v[1];
    return CMLB_OK;
}

int cmlb_inventories(cmlb_ctx* c, int32_t first, int32_t n, double* sums) {
    if (!c) return CMLB_EINVAL;
    if (!sums || first < 0 || n < 1 || first > c->n_sims - n)
        return fail(c, CMLB_EINVAL, "bad simulation range [%d, %d + %d) or null output", first,
                    first, n);
    int rc = launch_inventory(c, first, n, c->d_rows, c->d_inv);
    if (rc != CMLB_OK) return rc;
    HIP_TRY(c, hipMemcpyAsync(sums, c->d_inv, sizeof(double) * 2 * n, hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return CMLB_OK;
}

int cmlb_inventories_noalloc(cmlb_ctx* c, int32_t first, int32_t n, double* d_sums) {
    if (!c) return CMLB_EINVAL;
    if (!d_sums || (reinterpret_cast<uintptr_t>(d_sums) & 7) || first < 0 || n < 1 ||
        first > c->n_sims - n)
        return fail(c, CMLB_EINVAL,
                    "bad simulation range [%d, %d + %d) or null / misaligned device output",
                    first, first, n);
    const int64_t rows = rows_of_range(c, first, n);
    if (rows > SCRATCH_ROWS)
        return fail(c, CMLB_EINVAL,
                    "simulations [%d, %d) hold %lld rows, more than the %d rows of the scratch "
                    "array (CMLB_NOALLOC_MAX_ROWS)",
                    first, first + n, (long long)rows, SCRATCH_ROWS);
    if (!c->scratch)
        return fail(c, CMLB_EDEVICE, "device address of the scratch array unavailable: %s",
                    hipGetErrorString(c->scratch_err));
    return launch_inventory(c, first, n, static_cast<double*>(c->scratch), d_sums);
}

int cmlb_get_populations(cmlb_ctx* c, int32_t sim, double* f, double* h, double* g) {
    if (!c) return CMLB_EINVAL;
    if (!check_sim(c, sim)) return fail(c, CMLB_EINVAL, "bad simulation index");
    const SimDev& d = c->sims[sim];
    const int64_t plane = (int64_t)d.nx * d.ny;
    if (c->prec == CMLB_FP64)
        launch_decode<double>(c, sim);
    else if (c->prec == CMLB_FP32)
        launch_decode<float>(c, sim);
    else
        launch_decode<_Float16>(c, sim);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double* outs[3] = {f, h, g};
    for (int l = 0; l < c->nlat; ++l)
        if (outs[l])
            HIP_TRY(c, hipMemcpy(outs[l], c->d_stage + (int64_t)l * 9 * plane,
                                 sizeof(double) * 9 * plane, hipMemcpyDeviceToHost));
    return CMLB_OK;
}

int cmlb_set_populations(cmlb_ctx* c, int32_t sim, const double* f, const double* h,
                         const double* g) {
    if (!c) return CMLB_EINVAL;
    if (!check_sim(c, sim) || !f || !h || (c->nlat == 3 && !g))
        return fail(c, CMLB_EINVAL, "bad simulation index or population array");
    const SimDev& d = c->sims[sim];
    const int64_t plane = (int64_t)d.nx * d.ny;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const double* ins[3] = {f, h, g};
    for (int l = 0; l < c->nlat; ++l)
        HIP_TRY(c, hipMemcpy(c->d_stage + (int64_t)l * 9 * plane, ins[l], sizeof(double) * 9 * plane,
                             hipMemcpyHostToDevice));
    if (c->prec == CMLB_FP64)
        launch_encode<double>(c, sim);
    else if (c->prec == CMLB_FP32)
        launch_encode<float>(c, sim);
    else
        launch_encode<_Float16>(c, sim);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->inited[sim] = 1;
    return CMLB_OK;
}

int cmlb_set_step_count(cmlb_ctx* c, int64_t step) {
    if (!c || step < 0) return CMLB_EINVAL;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int64_t v[2] = {step, step};
    HIP_TRY(c, hipMemcpy(c->d_step, v, sizeof(v), hipMemcpyHostToDevice));
    c->step = step;
    return CMLB_OK;
}

int cmlb_fault_flags(cmlb_ctx* c, int32_t sim, int32_t* flags) {
    if (!c || !flags) return CMLB_EINVAL;
    if (!check_sim(c, sim)) return fail(c, CMLB_EINVAL, "bad simulation index");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(flags, c->d_fault + sim, sizeof(int32_t), hipMemcpyDeviceToHost));
    return CMLB_OK;
}

int cmlb_synchronize(cmlb_ctx* c) {
    if (!c) return CMLB_EINVAL;
    return sync_and_check(c);
}

int cmlb_set_tile_shape(cmlb_ctx* c, int32_t width, int32_t rows) {
    if (!c) return CMLB_EINVAL;
    if ((width == 0) != (rows == 0))
        return fail(c, CMLB_EINVAL, "tile width and rows must both be 0 or both set");
    if (width != 0 && !shape_of(c->prec, width, rows, nullptr))
        return fail(c, CMLB_EINVAL, "tile shape %dx%d not supported", width, rows);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->tile_w = width;
    c->tile_rows = rows;
    return build_tiles(c);
}

int cmlb_set_tile_rows(cmlb_ctx* c, int32_t rows) {
    if (!c) return CMLB_EINVAL;
    return cmlb_set_tile_shape(c, rows ? 64 : 0, rows);
}

int cmlb_launch_options(const cmlb_ctx* c, int32_t* shapes, int32_t cap) {
    if (!c || (!shapes && cap > 0)) return CMLB_EINVAL;
    const Shape* t = c->prec == CMLB_FP64 ? SHAPES_64 : SHAPES_32;
    const int n = c->prec == CMLB_FP64 ? N_SHAPES_64 : N_SHAPES_32;
    for (int i = 0; i < n && 2 * i + 1 < cap; ++i) {
        shapes[2 * i] = t[i].width;
        shapes[2 * i + 1] = t[i].rows;
    }
    return n;
}

int cmlb_set_use_graph(cmlb_ctx* c, int32_t on) {
    if (!c) return CMLB_EINVAL;
    c->use_graph = on ? 1 : 0;
    return CMLB_OK;
}

int cmlb_set_xcd_remap(cmlb_ctx* c, int32_t on) {
    if (!c) return CMLB_EINVAL;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->xcd_remap = on ? 1 : 0;
    drop_graphs(c);
    return CMLB_OK;
}

// Autotuner: every (tile shape, store policy) pair advances the context's
// own simulations by `steps` direct launches, timed with HIP events, each
// trial starting from the same saved state; the fastest pair is kept and the
// state restored, so the run continues bitwise as if no trial had happened.
int cmlb_autotune(cmlb_ctx* c, int32_t steps, int32_t* width, int32_t* rows, int32_t* policy) {
    if (!c || steps < 1 || steps > 100000) return CMLB_EINVAL;
    for (int s = 0; s < c->n_sims; ++s)
        if (!c->inited[s]) return fail(c, CMLB_ESTATE, "simulation %d not initialised", s);
    if (c->fault_seen) return fail(c, CMLB_ERANGE, "a fault flag was raised earlier");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int cur0 = c->cur;
    const int64_t step0 = c->step;
    const int w0 = c->tile_w, r0 = c->tile_rows, p0 = c->store_policy;
    int64_t dstep[2];
    std::vector<int32_t> fault(c->n_sims);
    HIP_TRY(c, hipMemcpy(dstep, c->d_step, sizeof(dstep), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(fault.data(), c->d_fault, sizeof(int32_t) * c->n_sims,
                         hipMemcpyDeviceToHost));
    void* save = nullptr;
    if (hipMalloc(&save, c->pop_bytes) != hipSuccess)
        return fail(c, CMLB_ENOMEM, "no device memory for the autotuner's state copy");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = CMLB_OK;
    auto restore = [&]() -> int {
        c->cur = cur0;
        c->step = step0;
        HIP_TRY(c, hipMemcpyAsync(c->pop[cur0], save, c->pop_bytes, hipMemcpyDeviceToDevice,
                                  c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->d_step, dstep, sizeof(dstep), hipMemcpyHostToDevice,
                                  c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->d_fault, fault.data(), sizeof(int32_t) * c->n_sims,
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        return CMLB_OK;
    };
    const Shape* t = c->prec == CMLB_FP64 ? SHAPES_64 : SHAPES_32;
    const int n = c->prec == CMLB_FP64 ? N_SHAPES_64 : N_SHAPES_32;
    float best = 0.f;
    int bw = 0, br = 0, bp = 0;
    do {
        if (hipMemcpyAsync(save, c->pop[cur0], c->pop_bytes, hipMemcpyDeviceToDevice,
                           c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess ||
            hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            rc = fail(c, CMLB_EDEVICE, "autotuner set-up failed");
            break;
        }
        for (int i = 0; i < n && rc == CMLB_OK; ++i)
            for (int pol = 1; pol <= 2 && rc == CMLB_OK; ++pol) {
                c->tile_w = t[i].width;
                c->tile_rows = t[i].rows;
                c->store_policy = pol;
                if ((rc = build_tiles(c)) != CMLB_OK) break;
                // untimed: builds the graph the timed steps replay (when the
                // context uses graphs), so trials are timed as runs are
                if ((rc = cmlb_step(c, 2 * GRAPH_PAIRS + 2)) != CMLB_OK) break;
                if (hipEventRecord(e0, c->stream) != hipSuccess) { rc = CMLB_EDEVICE; break; }
                if ((rc = cmlb_step(c, steps)) != CMLB_OK) break;
                float ms = 0.f;
                if (hipEventRecord(e1, c->stream) != hipSuccess ||
                    hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    rc = fail(c, CMLB_EDEVICE, "autotuner timing failed");
                    break;
                }
                if (bw == 0 || ms < best) {
                    best = ms;
                    bw = t[i].width;
                    br = t[i].rows;
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
        c->tile_w = w0;
        c->tile_rows = r0;
        c->store_policy = p0;
        (void)build_tiles(c);
        return rc;
    }
    (void)hipFree(save);
    c->tile_w = bw;
    c->tile_rows = br;
    c->store_policy = bp;
    if ((rc = build_tiles(c)) != CMLB_OK) return rc;
    if (width) *width = bw;
    if (rows) *rows = br;
    if (policy) *policy = bp;
    return CMLB_OK;
}

int cmlb_set_store_policy(cmlb_ctx* c, int32_t policy) {
    if (!c || policy < 0 || policy > 2) return CMLB_EINVAL;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->store_policy = policy;
    drop_graphs(c);
    return CMLB_OK;
}

int cmlb_set_tile_order(cmlb_ctx* c, int32_t group) {
    if (!c || group < 0) return CMLB_EINVAL;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->tile_group = group;
    return build_tiles(c);
}

int cmlb_launch_costs(int32_t blocks, int32_t iters, double* us_grid_sync, double* us_graph_node) {
    if (blocks < 1 || blocks > 1024 || iters < 16 || iters > 1000000 || (iters % 16) ||
        !us_grid_sync || !us_graph_node)
        return CMLB_EINVAL;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    float* sink = nullptr;
    int rc = CMLB_OK;
    auto ok = [&](hipError_t e) {
        if (e != hipSuccess && rc == CMLB_OK) rc = CMLB_EDEVICE;
        return rc == CMLB_OK;
    };
    do {
        if (!ok(hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) || !ok(hipEventCreate(&e0)) ||
            !ok(hipEventCreate(&e1)) || !ok(hipMalloc(&sink, sizeof(float) * blocks)))
            break;
        // (1) a cooperative launch whose workgroups meet at a grid barrier
        // `iters` times; the runtime refuses a grid that cannot be resident
        int32_t n = iters;
        void* args[] = {&n, &sink};
        if (!ok(hipLaunchCooperativeKernel((void*)cmlb::k_grid_sync_loop, dim3(blocks), dim3(256),
                                           args, 0, s)) ||
            !ok(hipStreamSynchronize(s)) || !ok(hipEventRecord(e0, s)) ||
            !ok(hipLaunchCooperativeKernel((void*)cmlb::k_grid_sync_loop, dim3(blocks), dim3(256),
                                           args, 0, s)) ||
            !ok(hipEventRecord(e1, s)) || !ok(hipEventSynchronize(e1)))
            break;
        float ms = 0.f;
        if (!ok(hipEventElapsedTime(&ms, e0, e1))) break;
        *us_grid_sync = 1e3 * ms / iters;
        // (2) a graph of 16 dependent launches of a kernel that does nothing,
        // replayed iters / 16 times: the per-step cost of the step graphs
        if (!ok(hipGraphCreate(&g, 0))) break;
        hipGraphNode_t prev = nullptr;
        for (int i = 0; i < 16 && rc == CMLB_OK; ++i) {
            hipKernelNodeParams np{};
            void* kargs[] = {&sink};
            np.func = (void*)cmlb::k_nothing;
            np.gridDim = dim3(blocks);
            np.blockDim = dim3(256);
            np.kernelParams = kargs;
            hipGraphNode_t node;
            if (!ok(hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &np)))
                break;
            prev = node;
        }
        if (rc != CMLB_OK || !ok(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0)) ||
            !ok(hipGraphLaunch(ge, s)) || !ok(hipStreamSynchronize(s)) ||
            !ok(hipEventRecord(e0, s)))
            break;
        for (int i = 0; i < iters / 16 && rc == CMLB_OK; ++i) ok(hipGraphLaunch(ge, s));
        if (rc != CMLB_OK || !ok(hipEventRecord(e1, s)) || !ok(hipEventSynchronize(e1)) ||
            !ok(hipEventElapsedTime(&ms, e0, e1)))
            break;
        *us_graph_node = 1e3 * ms / iters;
    } while (false);
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    if (sink) (void)hipFree(sink);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    return rc;
}

int cmlb_copy(const void* src, void* dst, int64_t bytes, int32_t nontemporal, void* hip_stream) {
    if (!src || !dst || bytes < 0 || (bytes & 15) || (reinterpret_cast<uintptr_t>(src) & 15) ||
        (reinterpret_cast<uintptr_t>(dst) & 15) || (nontemporal != 0 && nontemporal != 1))
        return CMLB_EINVAL;
    const int64_t n4 = bytes / 16;
    if (n4 == 0) return CMLB_OK;
    const int64_t blocks = (n4 + 4 * 256 - 1) / (4 * 256);
    if (blocks > 0x7fffffff) return CMLB_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const auto* a = static_cast<const cmlb::f32x4*>(src);
    auto* b = static_cast<cmlb::f32x4*>(dst);
    if (nontemporal)
        hipLaunchKernelGGL(cmlb::k_copy<true>, dim3((unsigned)blocks), dim3(256), 0, s, a, b, n4);
    else
        hipLaunchKernelGGL(cmlb::k_copy<false>, dim3((unsigned)blocks), dim3(256), 0, s, a, b, n4);
    return hipGetLastError() == hipSuccess ? CMLB_OK : CMLB_EDEVICE;
}

int cmlb_copy_planes(const void* src, void* dst, int64_t plane_bytes, int32_t planes,
                     int32_t nontemporal, void* hip_stream) {
    if (!src || !dst || plane_bytes < 0 || (plane_bytes & 15) ||
        (reinterpret_cast<uintptr_t>(src) & 15) || (reinterpret_cast<uintptr_t>(dst) & 15) ||
        (planes != 9 && planes != 27) || (nontemporal != 0 && nontemporal != 1))
        return CMLB_EINVAL;
    const int64_t n4 = plane_bytes / 16;
    if (n4 == 0) return CMLB_OK;
    const int64_t blocks = (n4 + 255) / 256;
    if (blocks > 0x7fffffff) return CMLB_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const auto* a = static_cast<const cmlb::f32x4*>(src);
    auto* b = static_cast<cmlb::f32x4*>(dst);
    const dim3 g((unsigned)blocks), t(256);
    if (planes == 9 && nontemporal)
        hipLaunchKernelGGL((cmlb::k_copy_planes<9, true>), g, t, 0, s, a, b, n4);
    else if (planes == 9)
        hipLaunchKernelGGL((cmlb::k_copy_planes<9, false>), g, t, 0, s, a, b, n4);
    else if (nontemporal)
        hipLaunchKernelGGL((cmlb::k_copy_planes<27, true>), g, t, 0, s, a, b, n4);
    else
        hipLaunchKernelGGL((cmlb::k_copy_planes<27, false>), g, t, 0, s, a, b, n4);
    return hipGetLastError() == hipSuccess ? CMLB_OK : CMLB_EDEVICE;
}

int64_t cmlb_step_count(const cmlb_ctx* c) { return c ? c->step : -1; }
int32_t cmlb_num_sims(const cmlb_ctx* c) { return c ? c->n_sims : 0; }
const char* cmlb_last_error(const cmlb_ctx* c) { return c ? c->err.c_str() : "null context"; }

void cmlb_destroy(cmlb_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    release(c);
    delete c;
}

}  // extern "C"
