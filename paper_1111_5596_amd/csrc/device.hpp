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
// largest magnitude m (m = f 2^e, 0.5 <= f < 1); kF16sZeroScale for an
// all-zero record.  Returns e (0 for zero; the caller stores
// f16s_scale(m, e)).
__device__ __forceinline__ int f16s_exponent(float m) {
    return m > 0.f ? __builtin_amdgcn_frexp_expf(m) : 0;
}
__device__ __forceinline__ float f16s_scale(float m, int e) {
    return m > 0.f ? __builtin_ldexpf(1.0f, e) : kF16sZeroScale;
}

// a * b + (float)h.x and a * b + (float)h.y in one rounding (the widening
// of a half is exact; the compiler forms v_fma_mix_f32).
__device__ __forceinline__ float fma_mix_lo(float a, float b, half2_t h) { return __builtin_fmaf(a, b, (float)h.x); }
__device__ __forceinline__ float fma_mix_hi(float a, float b, half2_t h) { return __builtin_fmaf(a, b, (float)h.y); }
// max(|a|, |b|, c) (v_max3_f32)
__device__ __forceinline__ float max3_abs(float a, float b, float c) {
    return __builtin_fmaxf(__builtin_fmaxf(__builtin_fabsf(a), __builtin_fabsf(b)), c);
}
// (half(x * s), half(y * s)); for s a power of two the products are exact,
// so this is the round-to-nearest-even FP16 of x * s and y * s.
__device__ __forceinline__ half2_t mul_to_half2(float x, float y, float s) {
    return half2_t{(_Float16)(x * s), (_Float16)(y * s)};
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

// These are plain code rather than inline assembly on purpose: the compiler
// inserts the wait states a VALU instruction needs after a v_dot2 that wrote
// one of its sources only for instructions it generated itself, not for
// inline assembly.

// Raw buffer access: one 128-bit resource per field (base address, no
// stride, full 32-bit range), a per-lane byte offset in a VGPR shared by all
// component planes, and the plane offset as a uniform (SGPR) operand.  This
// removes the 64-bit address arithmetic a flat load needs for every plane.
// Requires every accessed offset of the field to be below 4 GiB.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

// `p` must be the same for every lane of the wavefront (true for all the
// field bases the kernels address): it is read from the first lane so the
// resource lives in scalar registers.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* p) {
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    void* u = reinterpret_cast<void*>(((uint64_t)hi << 32) | lo);
    // word 3: 32-bit data format, the setting used for raw buffers on gfx9
    return __builtin_amdgcn_make_buffer_rsrc(u, (short)0, -1, 0x00020000);
}

__device__ __forceinline__ half2_t buf_load_h2(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return __builtin_bit_cast(half2_t, __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0));
}
__device__ __forceinline__ float buf_load_f32(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0));
}
__device__ __forceinline__ float2 buf_load_c32(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0));
}
__device__ __forceinline__ double2 buf_load_c64(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)so, 0));
}
__device__ __forceinline__ void buf_store_h2(half2_t v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, (int)vo, (int)so, 0);
}
__device__ __forceinline__ void buf_store_f32(float v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, (int)vo, (int)so, 0);
}
__device__ __forceinline__ void buf_store_c32(float2 v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, (int)vo, (int)so, 0);
}
__device__ __forceinline__ void buf_store_c64(double2 v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, v), r, (int)vo, (int)so, 0);
}

template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so);
template <>
__device__ __forceinline__ float2 bload<float2>(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return buf_load_c32(r, vo, so);
}
template <>
__device__ __forceinline__ double2 bload<double2>(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return buf_load_c64(r, vo, so);
}
template <>
__device__ __forceinline__ half2_t bload<half2_t>(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return buf_load_h2(r, vo, so);
}
template <>
__device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return buf_load_f32(r, vo, so);
}
__device__ __forceinline__ void bstore(float2 v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    buf_store_c32(v, r, vo, so);
}
__device__ __forceinline__ void bstore(double2 v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    buf_store_c64(v, r, vo, so);
}
__device__ __forceinline__ void bstore(half2_t v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    buf_store_h2(v, r, vo, so);
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    buf_store_f32(v, r, vo, so);
}

// Access to the rows of a tiled field (see common.hpp).  `so` is the byte
// offset of a site in row 0, tile_site_offset(tile bytes, sizeof(T), site);
// row r of that site is r * 64 * sizeof(T) bytes further.  The buffer path
// keeps one 32-bit per-lane offset per site and turns the row offsets into
// instruction immediates (needs the field below 4 GiB, checked on the host);
// the flat path uses 64-bit addresses.
template <typename T, bool BUF>
struct FieldRef {
    const char* base;
    __amdgpu_buffer_rsrc_t rsrc;
    __device__ __forceinline__ explicit FieldRef(const char* p) : base(p) {
        if constexpr (BUF) rsrc = buffer_rsrc(p);
    }
    // the row offset goes in the scalar offset operand (it is the same for
    // every lane): as part of the per-lane offset it would cost a vector add
    // per load, since the compiler cannot prove that sum free of wrap-around
    // and so will not fold it into the instruction's immediate offset
    __device__ __forceinline__ T load(int row, int64_t so) const {
        if constexpr (BUF)
            return bload<T>(rsrc, (uint32_t)so, (uint32_t)(row * 64 * (int)sizeof(T)));
        else
            return *reinterpret_cast<const T*>(base + so + (int64_t)row * 64 * (int64_t)sizeof(T));
    }
    __device__ __forceinline__ void store(T v, int row, int64_t so) const {
        if constexpr (BUF)
            bstore(v, rsrc, (uint32_t)so, (uint32_t)(row * 64 * (int)sizeof(T)));
        else
            *reinterpret_cast<T*>(const_cast<char*>(base) + so + (int64_t)row * 64 * (int64_t)sizeof(T)) = v;
    }
    // non-temporal store of a 4-byte value (see ChunkRef::store_stream)
    __device__ __forceinline__ void store_stream(T v, int row, int64_t so) const {
        static_assert(sizeof(T) == 4, "4-byte rows only");
        if constexpr (BUF)
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), rsrc, (int)(uint32_t)so,
                                                  row * 64 * 4, 2);
        else
            __builtin_nontemporal_store(v, reinterpret_cast<T*>(const_cast<char*>(base) + so + (int64_t)row * 64 * 4));
    }
};

// Access to the 16-byte chunks of a chunked field (see common.hpp): `so16` is
// tile_site_offset(tile bytes, 16, site); chunk q of that site is q * 1024
// bytes further.  Same addressing choices as FieldRef.
template <bool BUF>
struct ChunkRef {
    const char* base;
    __amdgpu_buffer_rsrc_t rsrc;
    __device__ __forceinline__ explicit ChunkRef(const char* p) : base(p) {
        if constexpr (BUF) rsrc = buffer_rsrc(p);
    }
    __device__ __forceinline__ u32x4_t load(int q, int64_t so16) const {
        if constexpr (BUF)
            return __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)(uint32_t)so16, q * 1024, 0);
        else
            return *reinterpret_cast<const u32x4_t*>(base + so16 + (int64_t)q * 1024);
    }
    // non-temporal load (cache policy nt): for data read once
    __device__ __forceinline__ u32x4_t load_stream(int q, int64_t so16) const {
        if constexpr (BUF)
            return __builtin_amdgcn_raw_buffer_load_b128(rsrc, (int)(uint32_t)so16, q * 1024, 2);
        else
            return __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(base + so16 + (int64_t)q * 1024));
    }
    __device__ __forceinline__ void store(u32x4_t v, int q, int64_t so16) const {
        if constexpr (BUF)
            __builtin_amdgcn_raw_buffer_store_b128(v, rsrc, (int)(uint32_t)so16, q * 1024, 0);
        else
            *reinterpret_cast<u32x4_t*>(const_cast<char*>(base) + so16 + (int64_t)q * 1024) = v;
    }
    // non-temporal store (cache policy nt): for results the kernel never
    // reads back, so that they do not push the records it still reads out
    // of the caches
    __device__ __forceinline__ void store_stream(u32x4_t v, int q, int64_t so16) const {
        if constexpr (BUF)
            __builtin_amdgcn_raw_buffer_store_b128(v, rsrc, (int)(uint32_t)so16, q * 1024, 2);
        else
            __builtin_nontemporal_store(v, reinterpret_cast<u32x4_t*>(const_cast<char*>(base) + so16 + (int64_t)q * 1024));
    }
};

template <typename T2>
struct Chunk {
    T2 v[16 / sizeof(T2)];
};

// Complex elements [E0, E0 + N) of a site of a chunked field (element e lies
// in chunk e / (16 / sizeof(T2))), one 16-byte load per chunk touched.
template <int E0, int N, bool STREAM = false, typename T2, bool BUF>
__device__ __forceinline__ void load_elems(const ChunkRef<BUF>& f, int64_t so16, T2* out) {
    constexpr int CE = 16 / sizeof(T2);
#pragma unroll
    for (int q = E0 / CE; q <= (E0 + N - 1) / CE; ++q) {
        const Chunk<T2> c = __builtin_bit_cast(Chunk<T2>, STREAM ? f.load_stream(q, so16) : f.load(q, so16));
#pragma unroll
        for (int j = 0; j < CE; ++j) {
            const int e = q * CE + j;
            if (e >= E0 && e < E0 + N) out[e - E0] = c.v[j];
        }
    }
}

// Store elements [0, N) of a site, N a multiple of the chunk size
// (STREAM: non-temporal stores).
template <int N, bool STREAM = false, typename T2, bool BUF>
__device__ __forceinline__ void store_elems(const ChunkRef<BUF>& f, int64_t so16, const T2* in) {
    constexpr int CE = 16 / sizeof(T2);
    static_assert(N % CE == 0, "whole chunks only");
#pragma unroll
    for (int q = 0; q < N / CE; ++q) {
        Chunk<T2> c;
#pragma unroll
        for (int j = 0; j < CE; ++j) c.v[j] = in[q * CE + j];
        if constexpr (STREAM)
            f.store_stream(__builtin_bit_cast(u32x4_t, c), q, so16);
        else
            f.store(__builtin_bit_cast(u32x4_t, c), q, so16);
    }
}

// Site offset in row 0 for elements of type T in tiles of `tb` bytes.
template <typename T>
__device__ __forceinline__ int64_t site_off(int32_t site, int64_t tb) {
    return (int64_t)(site >> 6) * tb + (int64_t)(site & 63) * (int64_t)sizeof(T);
}

// a.x b.x + a.y b.y in FP32 (v_dot2_f32_f16 with a zero accumulator)
__device__ __forceinline__ float dot2_zero(half2_t a, half2_t b) { return __builtin_amdgcn_fdot2(a, b, 0.f, false); }

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
