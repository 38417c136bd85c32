// Device helpers shared by the 2D (D2Q9) and 3D (D3Q27) step kernels:
// population storage through buffer descriptors in FP64, FP32 or binary16
// (stochastic rounding), the counter-based random words of that rounding,
// fast FP32 reciprocal / square root / logarithm, unbiased FP32 division by
// small constants, and coordinate folding.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cmlb {

template <class S>
struct Store {
    static constexpr bool scaled = false;
};
template <>
struct Store<_Float16> {
    static constexpr bool scaled = true;
};

// ---------------------------------------------------------------------------
// Storage access through buffer descriptors: the node offset in a VGPR and
// the direction's offset in the SGPR offset, so the loads and stores of a
// node share one address computation (`gload` reads through a plain 64-bit
// address instead, for paths whose offsets vary per load).  Out-of-range
// buffer accesses return 0 / are dropped by the hardware.  `load` returns
// the stored value in the compute type; `raw` returns it as a register word
// (binary16 zero-extended to 32 bits, one value per register) for `widen` to
// convert later, after the branches that issue the loads, so that a wave's
// loads stay in flight together (a conversion inside a branch waits for its
// load before the branch ends).
// ---------------------------------------------------------------------------
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, bytes, 0x00020000);
}

// Stores take a cache policy CP: 0 = default, CPOL_NT = non-temporal
// (streamed past the caches rather than kept in them).
constexpr int CPOL_NT = 2;

template <class S>
struct Buf;
template <>
struct Buf<double> {
    using word = double;
    static __device__ __forceinline__ double widen(word w) { return w; }
    static __device__ __forceinline__ double raw(__amdgpu_buffer_rsrc_t r, int vo, int so) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    }
    static __device__ __forceinline__ double load(__amdgpu_buffer_rsrc_t r, int vo, int so) {
        return raw(r, vo, so);
    }
    static __device__ __forceinline__ double gload(const char* p) {
        return *reinterpret_cast<const double*>(p);
    }
    template <int CP>
    static __device__ __forceinline__ void store(__amdgpu_buffer_rsrc_t r, int vo, int so, double v,
                                                 uint32_t) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, vo, so, CP);
    }
};
template <>
struct Buf<float> {
    using word = float;
    static __device__ __forceinline__ float widen(word w) { return w; }
    static __device__ __forceinline__ float raw(__amdgpu_buffer_rsrc_t r, int vo, int so) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    }
    static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, int vo, int so) {
        return raw(r, vo, so);
    }
    static __device__ __forceinline__ float gload(const char* p) {
        return *reinterpret_cast<const float*>(p);
    }
    template <int CP>
    static __device__ __forceinline__ void store(__amdgpu_buffer_rsrc_t r, int vo, int so, float v,
                                                 uint32_t) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, vo, so, CP);
    }
};
// binary16 storage: values widen exactly to FP32; stores round
// stochastically with gfx950's v_cvt_sr_f16_f32 (the top 13 bits of the
// random word decide the rounding direction; exactly representable values
// are kept).  Stochastic
// rounding keeps the per-step storage errors independent and unbiased, where
// round-to-nearest would repeat the same error every step at a quasi-steady
// node.
template <>
struct Buf<_Float16> {
    using word = uint32_t;
    static __device__ __forceinline__ float widen(word w) {
        return float(__builtin_bit_cast(_Float16, (unsigned short)w));
    }
    static __device__ __forceinline__ word raw(__amdgpu_buffer_rsrc_t r, int vo, int so) {
        return __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0);
    }
    static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, int vo, int so) {
        return float(__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0)));
    }
    static __device__ __forceinline__ float gload(const char* p) {
        return float(*reinterpret_cast<const _Float16*>(p));
    }
    template <int CP>
    static __device__ __forceinline__ void store(__amdgpu_buffer_rsrc_t r, int vo, int so, float v,
                                                 uint32_t rnd) {
        // the conversion writes the low half of its destination and keeps
        // the high half; passing v's own bits (dead after this) as that
        // destination lets the compiler convert in place
        const h16x2 h =
            __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(h16x2, v), v, rnd, false);
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, h[0]), r, vo, so,
                                              CP);
    }
};

// Counter-based random words for the stochastic rounding, from the
// MurmurHash3 32-bit finaliser fmix32.  A step has a key (the hash of the
// step number); a node's seed for that step is fmix32(node * 0x9E3779B9 +
// key), and its store to direction q of any lattice uses seed + q *
// 0x9E3779B9 (a Weyl sequence: one add per direction, shared by the node's
// three lattices; its top bits, the ones the conversion uses, are
// equidistributed).  The seed must be a hash of the (node, step) pair: the
// XOR fmix32(node) ^ key relates every node's words at consecutive steps by
// the same global XOR, and the rounding then drifts the inventories
// systematically (phi by 2.9e-3 over 5000 steps of a 256x128x128 drop),
// where a hashed pair leaves random-walk noise (1e-5).
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}
__device__ __forceinline__ uint32_t node_step_seed(uint32_t node, uint32_t step_key) {
    return fmix32(node * 0x9E3779B9u + step_key);
}
__device__ __forceinline__ constexpr uint32_t weyl(int k) { return (uint32_t)k * 0x9E3779B9u; }

// Fast approximate operations for the FP32 path (1-2 ulp), exact IEEE ones
// for FP64 (the FP64 path is checked against the oracle at 1e-12).
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_(double x) { return 1.0 / x; }
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
__device__ __forceinline__ float log_(float x) { return __logf(x); }
__device__ __forceinline__ double log_(double x) { return log(x); }

// x / D for a small integer D.  FP32 has no exact 1/9 or 1/36 (both round
// 7.45e-9 high): a product with the rounded reciprocal carries that bias in
// every result, and a scheme that divides by the lattice weights each step
// then gains or loses the divided quantity by 7.45e-9 per step.  One FMA
// residual step turns the product into the correctly rounded quotient
// (Markstein's correction), whose errors have no sign preference.
template <int D>
__device__ __forceinline__ float div_const(float x) {
    constexpr float r = 1.0f / D;
    const float q0 = x * r;
    const float e = __builtin_fmaf(-q0, float(D), x);
    return __builtin_fmaf(e, r, q0);
}

// Coordinate folding: periodic wrap, or mirror about the wall planes
// y = -1/2 and y = n - 1/2 (ghost row -1-k carries row k).
__device__ __forceinline__ int wrap_coord(int v, int n) {
    if (v >= 0 && v < n) return v;
    int m = v % n;
    return m < 0 ? m + n : m;
}
__device__ __forceinline__ int mirror_coord(int v, int n) {
    if (v >= 0 && v < n) return v;
    const int p = 2 * n;
    int m = v % p;
    if (m < 0) m += p;
    return m < n ? m : p - 1 - m;
}

}  // namespace cmlb
