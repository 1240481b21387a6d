// Device helpers: complex multiply-accumulate with explicit FMAs (so that
// every kernel variant rounds identically), half-precision record codec and
// site-geometry helpers for the checkerboard layout.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace qdpmi {

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

template <typename R>
struct Cplx;
template <>
struct Cplx<float> {
    using type = float2;
};
template <>
struct Cplx<double> {
    using type = double2;
};
template <typename R>
using cplx_t = typename Cplx<R>::type;

__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// acc += u * v
template <typename T2>
__device__ __forceinline__ void cmac(T2& acc, const T2& u, const T2& v) {
    acc.x = fmadd(u.x, v.x, acc.x);
    acc.x = fmadd(-u.y, v.y, acc.x);
    acc.y = fmadd(u.x, v.y, acc.y);
    acc.y = fmadd(u.y, v.x, acc.y);
}

// acc += conj(u) * v
template <typename T2>
__device__ __forceinline__ void cmac_conj(T2& acc, const T2& u, const T2& v) {
    acc.x = fmadd(u.x, v.x, acc.x);
    acc.x = fmadd(u.y, v.y, acc.x);
    acc.y = fmadd(u.x, v.y, acc.y);
    acc.y = fmadd(-u.y, v.x, acc.y);
}

// Scale factor of an F16S record: 2^e with e the binary exponent of the
// largest magnitude m (m = f 2^e, 0.5 <= f < 1); 1 for an all-zero record.
// Returns e (0 for zero).
__device__ __forceinline__ int f16s_exponent(float m) {
    return m > 0.f ? __builtin_amdgcn_frexp_expf(m) : 0;
}

__device__ __forceinline__ half2_t f16s_encode(float re, float im, int e) {
    half2_t q;
    q.x = (_Float16)__builtin_ldexpf(re, -e);
    q.y = (_Float16)__builtin_ldexpf(im, -e);
    return q;
}

__device__ __forceinline__ float2 f16s_decode(half2_t q, float scale) {
    return make_float2((float)q.x * scale, (float)q.y * scale);
}

// Neighbour indices of a checkerboard site in the three spatial directions.
struct SpatialNeighbours {
    int32_t fwd[3];
    int32_t bwd[3];
};

__device__ __forceinline__ SpatialNeighbours spatial_neighbours(const Geometry& g, int32_t s) {
    const int32_t Vh = (int32_t)g.Vh;
    const int32_t p = s >= Vh ? 1 : 0;
    const int32_t i = s - p * Vh;
    const int32_t Lxh = g.Lxh, Ly = g.L[1], Lz = g.L[2];
    const int32_t h = i % Lxh;
    const int32_t r = i / Lxh;
    const int32_t y = r % Ly;
    const int32_t r2 = r / Ly;
    const int32_t z = r2 % Lz;
    const int32_t t = r2 / Lz;
    const int32_t xodd = (p + y + z + t) & 1;
    const int32_t ob = (1 - p) * Vh;
    const int32_t row = i - h;
    SpatialNeighbours n;
    const int32_t hp = xodd ? (h + 1 == Lxh ? 0 : h + 1) : h;
    const int32_t hm = xodd ? h : (h == 0 ? Lxh - 1 : h - 1);
    n.fwd[0] = ob + row + hp;
    n.bwd[0] = ob + row + hm;
    const int32_t sy = Lxh;
    n.fwd[1] = ob + i + (y == Ly - 1 ? -(Ly - 1) * sy : sy);
    n.bwd[1] = ob + i + (y == 0 ? (Ly - 1) * sy : -sy);
    const int32_t sz = Lxh * Ly;
    n.fwd[2] = ob + i + (z == Lz - 1 ? -(Lz - 1) * sz : sz);
    n.bwd[2] = ob + i + (z == 0 ? (Lz - 1) * sz : -sz);
    return n;
}

// XCD-aware block order: the hardware deals workgroups to the 8 XCDs round
// robin; this maps them so each XCD works through one contiguous range of
// logical blocks (its L2 then sees neighbouring sites).  Requires the grid
// to be padded to a multiple of 8; returns a logical index in [0, grid).
__device__ __forceinline__ int64_t xcd_logical_block(int64_t b, int64_t grid) {
    const int64_t per = grid >> 3;
    return (b & 7) * per + (b >> 3);
}

}  // namespace qdpmi
