// D3Q19 lattice constants and population storage formats for the gfx950 kernels.
//
// Velocity order used by this library: rest; +-x, +-y, +-z; then the twelve
// face diagonals as opposite pairs (xy, xz, yz).  Weights 1/3, 1/18, 1/36 by
// |c|^2 = 0, 1, 2, so that c_s^2 = 1/3, which is what the 3, 9/2 and 3/2
// coefficients of the equilibrium in Sec. 2 Eq. 8 of arXiv 2112.09972 assume.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sclbm.h"

// Debug build (SCLBM_DEBUG_FILL=1, the library's debug variant): the step kernels
// overwrite the LDS slots they are about to fill with NaN at every plane, so that
// a read of a cell no thread wrote for that plane turns into NaN populations.
#ifndef SCLBM_DEBUG_FILL
#define SCLBM_DEBUG_FILL 0
#endif

namespace sclbm {

constexpr bool kDebugFill = SCLBM_DEBUG_FILL != 0;

// Quiet-NaN bit patterns of the stored formats (debug fill).
template <typename T>
__device__ __forceinline__ T nan_bits(int prec) {
    if constexpr (sizeof(T) == 8) return T(0x7ff8000000000000ull);
    if constexpr (sizeof(T) == 2) return T(prec == SCLBM_BF16DEV ? 0x7fc0u : 0x7e00u);
    return T(prec == SCLBM_BF16DEV ? 0x7fc0u : (prec == SCLBM_F16DEV ? 0x7e00u : 0x7fc00000u));
}

// Fill n elements of an LDS array with `v`, all threads of the workgroup taking part.
template <typename T>
__device__ __forceinline__ void lds_fill(T *p, int n, T v, int tid, int nthreads) {
    for (int i = tid; i < n; i += nthreads) p[i] = v;
}

constexpr int Q = 19;

__host__ __device__ constexpr int cx_of(int i) {
    constexpr int v[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return v[i];
}
__host__ __device__ constexpr int cy_of(int i) {
    constexpr int v[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return v[i];
}
__host__ __device__ constexpr int cz_of(int i) {
    constexpr int v[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return v[i];
}
// Run-time lookups of the same table (for loops that are deliberately not
// unrolled): 2-bit codes per direction, 1 -> +1, 3 -> -1, 0 -> 0.
__host__ __device__ constexpr uint64_t pack_codes(int axis) {
    uint64_t p = 0;
    for (int i = 0; i < Q; ++i) {
        const int c = axis == 0 ? cx_of(i) : (axis == 1 ? cy_of(i) : cz_of(i));
        p |= uint64_t(c == 0 ? 0 : (c > 0 ? 1 : 3)) << (2 * i);
    }
    return p;
}
__device__ __forceinline__ int c_rt(int axis, int i) {
    const uint64_t p = axis == 0 ? pack_codes(0) : (axis == 1 ? pack_codes(1) : pack_codes(2));
    const int code = int((p >> (2 * i)) & 3);
    return code == 0 ? 0 : (code == 1 ? 1 : -1);
}

template <typename R>
__host__ __device__ constexpr R w_of(int i) {
    return i == 0 ? R(1) / R(3) : (i < 7 ? R(1) / R(18) : R(1) / R(36));
}

// Storage formats.  S is what lives in HBM, W the type a loaded population is
// held in registers (exactly representable from S), R the arithmetic type.
// FP32 storage computes in FP32 (SCLBM_F32) or in FP64 (SCLBM_F32D).  The
// FP32-rounded lattice weights do not sum to one (1 + 3e-8), so a single-rate
// collision in FP32 written population by population would create or destroy
// that much mass at every node and step (2e-5 density error after 500 steps of
// the droplet box); the step kernel therefore lets the rest population close
// the mass balance, rho minus the other eighteen post-collision values, which
// is the same update in exact arithmetic.  With FP64 arithmetic the only
// rounding is the storage's (1.1e-7 to 2.3e-7 after 500 steps of the droplet
// box at tau = 1, 3 and (0.8, 1.4), against 6.7e-7, 2.2e-5 and 3.8e-6 in FP32
// arithmetic; the tau = 3 run, with spurious currents of order 0.1, amplifies
// the extra roundings most).
// The deviation formats hold d_i = f_i / (w_i rho_ref(x)) - 1 in 16 bits with FP32
// arithmetic, rho_ref(x) being the node's own density one step earlier, kept
// per node and component in FP16 (DEV = true).  A constant reference fails in
// a two-phase box: the minority component inside the other phase deviates from
// w_i rho_ref by as much as the population itself (2.8e-2 density error after
// 500 steps of the 32^3 droplet box in FP16, 0.31 in BF16).
// Raw buffer access (CDNA buffer instructions): a 128-bit descriptor per
// population array in SGPRs, a uniform byte offset per direction (SGPR) and one
// 32-bit byte offset per lane.  Word 3 = 0x00020000 is the raw 32-bit-element
// layout of the gfx9 family.
using rsrc_t = __amdgpu_buffer_rsrc_t;
// Cache policy of the population stores: non-temporal (streaming).  Every
// population is written once per step and read only in the next launch; keeping
// the stores out of L2's working set leaves it to the rows that neighbouring
// tiles read again (measured: 12 % fewer HBM reads, 3 % faster step).
constexpr int kStoreNT = 2;
// The same hint on the loads of rows that no other workgroup reads (interior
// rows of a tile holding whole rows, on planes inside its z-chunk): they are read
// once per step, and streaming them leaves L2 to the rows that are read twice.
constexpr int kLoadNT = 2;
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, int(bytes), 0x00020000);
}

// Relative deviation (v - wref) / wref that the 16-bit formats store: it keeps
// the formats' relative precision at every size of deviation (an absolute
// deviation below 6e-5 would fall into FP16's subnormal range, whose spacing of
// 6e-8 is 1e-5 of a minority-phase population).  The reader rebuilds
// wref (1 + d); any consistent reciprocal will do.
__device__ __forceinline__ float rel_dev(float v, float wref) { return (v - wref) * __builtin_amdgcn_rcpf(wref); }

template <int P>
struct Prec;
template <>
struct Prec<SCLBM_F64> {
    static constexpr bool DEV = false;
    using S = double;
    using W = double;
    using R = double;
    using D = double;  // densities of the force stencil
    static __device__ __forceinline__ W load(const S *p, R /*wref*/) { return *p; }
    static __device__ __forceinline__ void store(S *p, R v, R /*wref*/) { *p = v; }
    static __device__ __forceinline__ W bload(rsrc_t r, uint32_t vo, uint32_t so, R /*wref*/) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    }
    using B = uint64_t;  // stored bits
    using L = uint64_t;  // raw loaded word
    template <int AUX = 0>
    static __device__ __forceinline__ L bload_raw(rsrc_t r, uint32_t vo, uint32_t so) {
        return __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, AUX));
    }
    static __device__ __forceinline__ W dec(L raw, R /*wref*/) { return __builtin_bit_cast(double, raw); }
    static __device__ __forceinline__ B enc(R v, R /*wref*/) { return __builtin_bit_cast(uint64_t, v); }
    static __device__ __forceinline__ void bstore_bits(rsrc_t r, uint32_t vo, uint32_t so, B b) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, b), r, vo, so, kStoreNT);
    }
    static __device__ __forceinline__ void bstore(rsrc_t r, uint32_t vo, uint32_t so, R v, R wref) {
        bstore_bits(r, vo, so, enc(v, wref));
    }
};
// FP32 storage; RT the arithmetic type (FP32 for SCLBM_F32, FP64 for SCLBM_F32D).
template <typename RT>
struct PrecF32 {
    static constexpr bool DEV = false;
    using S = float;
    using W = float;
    using R = RT;
    using D = double;
    static __device__ __forceinline__ W load(const S *p, R /*wref*/) { return *p; }
    static __device__ __forceinline__ void store(S *p, R v, R /*wref*/) { *p = float(v); }
    static __device__ __forceinline__ W bload(rsrc_t r, uint32_t vo, uint32_t so, R /*wref*/) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    }
    using B = uint32_t;
    using L = uint32_t;
    template <int AUX = 0>
    static __device__ __forceinline__ L bload_raw(rsrc_t r, uint32_t vo, uint32_t so) {
        return __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, AUX);
    }
    static __device__ __forceinline__ W dec(L raw, R /*wref*/) { return __builtin_bit_cast(float, raw); }
    static __device__ __forceinline__ B enc(R v, R /*wref*/) { return __builtin_bit_cast(uint32_t, float(v)); }
    static __device__ __forceinline__ void bstore_bits(rsrc_t r, uint32_t vo, uint32_t so, B b) {
        __builtin_amdgcn_raw_buffer_store_b32(b, r, vo, so, kStoreNT);
    }
    static __device__ __forceinline__ void bstore(rsrc_t r, uint32_t vo, uint32_t so, R v, R wref) {
        bstore_bits(r, vo, so, enc(v, wref));
    }
};
template <>
struct Prec<SCLBM_F32> : PrecF32<float> {};
template <>
struct Prec<SCLBM_F32D> : PrecF32<double> {};
// The deviation formats as the auxiliary kernels (initialisation, fields,
// moments) read and write them, one population at a time; the step kernel
// (k_step_dev) has its own arithmetic on the stored deviations.
template <>
struct Prec<SCLBM_F16DEV> {
    static constexpr bool DEV = true;
    using S = __half;
    using W = float;
    using R = float;
    static __device__ __forceinline__ W load(const S *p, R wref) { return wref + wref * __half2float(*p); }
    static __device__ __forceinline__ void store(S *p, R v, R wref) { *p = __float2half_rn(rel_dev(v, wref)); }
};
template <>
struct Prec<SCLBM_BF16DEV> {
    static constexpr bool DEV = true;
    using S = __hip_bfloat16;
    using W = float;
    using R = float;
    static __device__ __forceinline__ W load(const S *p, R wref) { return wref + wref * __bfloat162float(*p); }
    static __device__ __forceinline__ void store(S *p, R v, R wref) { *p = __float2bfloat16(rel_dev(v, wref)); }
};

// Per-node reference densities of the deviation formats (FP16; only their
// consistency between writer and reader matters, not their precision).
__device__ __forceinline__ float ref_load(const __half *p) { return __half2float(*p); }
__device__ __forceinline__ float ref_round(float v) { return __half2float(__float2half_rn(v)); }
__device__ __forceinline__ void ref_store(__half *p, float v) { *p = __float2half_rn(v); }

// Population layout within one box of N nodes, by element of the format's stored
// type S: e is the row-blocked index ((z ny + y) 19 + i) nx + x of direction i at a
// node.  FP64 and FP32 keep one array per component, [component][z][y][i][x]; the
// deviation formats keep both components of (node, i) side by side in one 32-bit
// word, A first: [z][y][i][x][component].  Their reference densities likewise,
// [node][component].
template <int P>
__host__ __device__ __forceinline__ int64_t pop_index(int64_t N, int64_t e, int s) {
    if constexpr (Prec<P>::DEV) return 2 * e + s;
    else return int64_t(s) * Q * N + e;
}
__host__ __device__ __forceinline__ int64_t ref_index(int64_t k, int s) { return 2 * k + s; }

inline bool is_dev(int prec) { return prec == SCLBM_F16DEV || prec == SCLBM_BF16DEV; }

inline size_t elem_bytes(int prec) {
    switch (prec) {
        case SCLBM_F64: return 8;
        case SCLBM_F32:
        case SCLBM_F32D: return 4;
        default: return 2;
    }
}

// Second-order equilibrium of Sec. 2 Eq. 8 for direction i.
template <typename R>
__device__ __forceinline__ R equilibrium(int i, R rho, R ux, R uy, R uz, R usq) {
    const R cu = R(cx_of(i)) * ux + R(cy_of(i)) * uy + R(cz_of(i)) * uz;
    return w_of<R>(i) * rho * (R(1) + R(3) * cu + R(4.5) * cu * cu - R(1.5) * usq);
}

}  // namespace sclbm
