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

namespace sclbm {

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
template <typename R>
__host__ __device__ constexpr R w_of(int i) {
    return i == 0 ? R(1) / R(3) : (i < 7 ? R(1) / R(18) : R(1) / R(36));
}

// Storage formats.  S is what lives in HBM, W the type a loaded population is
// held in registers (exactly representable from S), R the arithmetic type.
// FP32 storage computes in FP64: on gfx950 the FP64 vector rate equals the
// unpacked FP32 rate, and FP32 collide arithmetic accumulates cancellation error
// in the moments and the non-equilibrium part (about 100x the storage
// rounding after 500 steps of the droplet box).
// The deviation formats hold d_i = f_i - w_i rho_ref in 16 bits with FP32
// arithmetic; the reference density of each component is a context constant.
template <int P>
struct Prec;
template <>
struct Prec<SCLBM_F64> {
    using S = double;
    using W = double;
    using R = double;
    static __device__ __forceinline__ W load(const S *p, R /*wref*/) { return *p; }
    static __device__ __forceinline__ void store(S *p, R v, R /*wref*/) { *p = v; }
};
template <>
struct Prec<SCLBM_F32> {
    using S = float;
    using W = float;
    using R = double;
    static __device__ __forceinline__ W load(const S *p, R /*wref*/) { return *p; }
    static __device__ __forceinline__ void store(S *p, R v, R /*wref*/) { *p = float(v); }
};
template <>
struct Prec<SCLBM_F16DEV> {
    using S = __half;
    using W = float;
    using R = float;
    static __device__ __forceinline__ W load(const S *p, R wref) { return wref + __half2float(*p); }
    static __device__ __forceinline__ void store(S *p, R v, R wref) { *p = __float2half_rn(v - wref); }
};
template <>
struct Prec<SCLBM_BF16DEV> {
    using S = __hip_bfloat16;
    using W = float;
    using R = float;
    static __device__ __forceinline__ W load(const S *p, R wref) { return wref + __bfloat162float(*p); }
    static __device__ __forceinline__ void store(S *p, R v, R wref) { *p = __float2bfloat16(v - wref); }
};

inline size_t elem_bytes(int prec) {
    switch (prec) {
        case SCLBM_F64: return 8;
        case SCLBM_F32: return 4;
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
