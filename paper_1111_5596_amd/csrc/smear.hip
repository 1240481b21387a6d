// Jacobi smearing on gfx950: the hot loop of source and sink smearing
// (SRC / SNK, section 5 and Figure 4 of the paper).
//
//   psi_{k+1}(x) = psi_k(x) + kappa sum_{i=0,1,2} [ U_i(x) psi_k(x+i)
//                                                + U_i(x-i)^dagger psi_k(x-i) ]
//
// One thread updates one site for a group of columns; the six links of the
// site stay in registers and are reused by every column and spin, so the
// 12-column update reads each link once from memory.  The 3x3 complex
// mat-vecs run on the vector ALUs (there is no dense contraction to give to
// the matrix cores).  F16S storage keeps links and spinors as half2 with a
// per-record FP32 scale; products use v_dot2_f32_f16 (two half products
// accumulated in FP32) and the per-term scales are applied in FP32.
//
// Every launch shape (sites per block, column groups, XCD mapping), the
// single-lattice and the multi-lattice kernels, graph replay and eager
// launches run the same per-site code, so they produce bitwise-identical
// results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "device.hpp"
#include "internal.hpp"

namespace qdpmi {

struct SmearJob {
    Geometry g;
    const char* gauge;
    const char* src[12];
    char* dst[12];
    int32_t ncols;
    int32_t pad;
};

struct SmearLaunch {
    int64_t site_begin;  // first checkerboard site of the pass
    int64_t site_count;  // sites of the pass
    int64_t nlogical;    // logical blocks (grid may be padded to 8)
    int32_t site_waves;  // wavefronts of sites per block
    int32_t col_groups;  // column groups per site
    int32_t xcd;         // XCD-aware block mapping
    int32_t interleave;  // whole lattice: block 2b = even tile b, 2b+1 = odd tile b
    int32_t zstride;     // > 0: the waves of a block take 64-site tiles zstride apart
    int32_t xcd_group;   // xcd = 2: logical blocks per group kept on one XCD
    int32_t one_item;    // multi-lattice kernel: block b takes work item b only
    int32_t bands;       // LDS-window kernel: y bands walked one after another (1 = none)
    int32_t pad2;
    double kappa;
};

// ---------------------------------------------------------------------------
// Memory access of the per-site updates.  BUF = true: raw buffer loads with
// one byte offset per neighbour site shared by every component row (needs
// every field below 4 GiB); BUF = false: flat 64-bit addresses.  Both feed
// the same arithmetic, so they produce identical bits.
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Per-site update, FP64 / FP32 storage (arithmetic in the storage type)
// ---------------------------------------------------------------------------

template <typename R, bool BUF>
__device__ __forceinline__ void site_update_real(const SmearJob& job, int32_t s, int c0, int c1,
                                                 R kappa) {
    using T2 = cplx_t<R>;
    const SpatialNeighbours nb = spatial_neighbours(job.g, s);
    constexpr int PREC = sizeof(R) == 8 ? QDP_F64 : QDP_F32;
    const int64_t tbu = tile_bytes(4, 9, PREC), tbc = tile_bytes(1, 12, PREC);
    const ChunkRef<BUF> U(job.gauge);
    // 16-byte-chunk site offsets: links at x and x - i, column values at x, x + i, x - i
    const int64_t us = tile_site_offset(tbu, 16, s);
    const int64_t cs = tile_site_offset(tbc, 16, s);
    int64_t ub_off[3], cf[3], cb[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        ub_off[i] = tile_site_offset(tbu, 16, nb.bwd[i]);
        cf[i] = tile_site_offset(tbc, 16, nb.fwd[i]);
        cb[i] = tile_site_offset(tbc, 16, nb.bwd[i]);
    }

    // links: elements 9 i .. 9 i + 8 of the gauge record are U_i
    T2 uf[3][9], ub[3][9];
    {
        T2 u[27];
        load_elems<0, 27>(U, us, u);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 9; ++k) uf[i][k] = u[9 * i + k];
    }
    load_elems<0, 9>(U, ub_off[0], ub[0]);
    load_elems<9, 9>(U, ub_off[1], ub[1]);
    load_elems<18, 9>(U, ub_off[2], ub[2]);

    for (int c = c0; c < c1; ++c) {
        const ChunkRef<BUF> src(job.src[c]);
        T2 acc[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = T2{0, 0};
        // Two load batches per column (the three forward neighbours, then the
        // three backward neighbours and the site itself), each requested in
        // full before its arithmetic: two waits on memory per column while
        // the links stay in registers.
        T2 v[3][12];
#pragma unroll
        for (int i = 0; i < 3; ++i) load_elems<0, 12>(src, cf[i], v[i]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) cmac(acc[3 * sp + a], uf[i][3 * a + b], v[i][3 * sp + b]);
        T2 own[12];
#pragma unroll
        for (int i = 0; i < 3; ++i) load_elems<0, 12>(src, cb[i], v[i]);
        load_elems<0, 12, true>(src, cs, own);  // read once: non-temporal
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) cmac_conj(acc[3 * sp + a], ub[i][3 * b + a], v[i][3 * sp + b]);
        T2 out[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            out[k] = own[k];
            out[k].x = fmadd(kappa, acc[k].x, out[k].x);
            out[k].y = fmadd(kappa, acc[k].y, out[k].y);
        }
        store_elems<12, true>(ChunkRef<BUF>(job.dst[c]), cs, out);
    }
}

// ---------------------------------------------------------------------------
// Per-site update, F16S storage (FP32 arithmetic)
// ---------------------------------------------------------------------------

// a.x b.x + a.y b.y + c in FP32 (v_dot2_f32_f16 or its two-operand form
// v_dot2c_f32_f16, the same operation).  Never inline assembly: a VALU
// instruction that reads a v_dot2 result needs wait states after it, which
// the compiler inserts only for instructions it generated itself.
__device__ __forceinline__ float dot2(half2_t a, half2_t b, float c) { return __builtin_amdgcn_fdot2(a, b, c, false); }

// The F16S update of one site and column, shared by every kernel variant so
// that all of them produce the same bits.  The six hop terms are taken in the
// fixed order z forward, z backward, y forward, y backward, x forward, x
// backward (hop h: direction kHopDir[h], backward when h is odd).
constexpr int kHopDir[6] = {2, 2, 1, 1, 0, 0};

// The links of one site in the two half2 forms the products need, per hop:
// forward link u = U_i(x):        re(u v) = (u.x, -u.y).v  im(u v) = (u.y, u.x).v
// backward link w = U_i(x - i)^T: re(w* v) = (w.x, w.y).v   im(w* v) = (-w.y, w.x).v
// element [3 a + b] of a hop multiplies colour b of the neighbour into colour
// a of the result (the backward link stored transposed), with the record's
// FP32 scale.
struct F16sLinks {
    half2_t re[6][9], im[6][9];
    float s[6];
};

template <bool BUF>
__device__ __forceinline__ void load_links_f16s(const char* gauge, int32_t s, const SpatialNeighbours& nb,
                                                F16sLinks& L) {
    const int64_t tbu = tile_bytes(4, 9, QDP_F16S);
    const ChunkRef<BUF> U(gauge);
    const FieldRef<float, BUF> Us(gauge);
    const int64_t us = tile_site_offset(tbu, 16, s), us4 = site_off<float>(s, tbu);
    half2_t u[27], w[3][9];
    load_elems<0, 27>(U, us, u);
    load_elems<0, 9>(U, tile_site_offset(tbu, 16, nb.bwd[0]), w[0]);
    load_elems<9, 9>(U, tile_site_offset(tbu, 16, nb.bwd[1]), w[1]);
    load_elems<18, 9>(U, tile_site_offset(tbu, 16, nb.bwd[2]), w[2]);
#pragma unroll
    for (int h = 0; h < 6; ++h) {
        const int i = kHopDir[h];
        if (h & 1) {
            L.s[h] = Us.load(36 + i, site_off<float>(nb.bwd[i], tbu));
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const half2_t ww = w[i][3 * b + a];
                    L.re[h][3 * a + b] = ww;
                    L.im[h][3 * a + b] = half2_t{(_Float16)(-ww.y), ww.x};
                }
        } else {
            L.s[h] = Us.load(36 + i, us4);
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const half2_t uu = u[9 * i + k];
                L.re[h][k] = half2_t{uu.x, (_Float16)(-uu.y)};
                L.im[h][k] = half2_t{uu.y, uu.x};
            }
        }
    }
}

// Common scale of the six hop terms.  Hop h multiplies a link record (scale
// a_h) and a neighbour record (scale b_h), both powers of two; with M the
// largest p_h = a_h b_h the neighbour's halves are multiplied by p_h / M <= 1
// (exact in FP16 down to its subnormal range: only terms below 2^-24 of the
// largest lose bits, as they would in an FP32 sum), so that every product of
// halves goes, exactly formed, into one FP32 sum per component.
struct F16sHopScale {
    float M;
    half2_t f[6];
};
__device__ __forceinline__ F16sHopScale hop_scale_f16s(const F16sLinks& L, const float nsc[6]) {
    F16sHopScale H;
    float p[6];
#pragma unroll
    for (int h = 0; h < 6; ++h) p[h] = L.s[h] * nsc[h];
    H.M = fmaxf(fmaxf(fmaxf(p[0], p[1]), fmaxf(p[2], p[3])), fmaxf(p[4], p[5]));
    const int eM = __builtin_amdgcn_frexp_expf(H.M);  // M = 2^(eM - 1)
#pragma unroll
    for (int h = 0; h < 6; ++h) {
        const _Float16 f = (_Float16)__builtin_ldexpf(p[h], 1 - eM);
        H.f[h] = half2_t{f, f};
    }
    return H;
}

// acc (+)= hop h of (1/M) [U psi]: the neighbour record v (as stored) brought
// to the common scale, then three products per result component.
template <int H>
__device__ __forceinline__ void hop_accumulate_f16s(float2 acc[12], const F16sLinks& L, const F16sHopScale& S,
                                                    const half2_t v_in[12]) {
    half2_t v[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = v_in[k] * S.f[H];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float re = acc[3 * sp + a].x, im = acc[3 * sp + a].y;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                if (H == 0 && b == 0) {
                    re = dot2_zero(L.re[H][3 * a], v[3 * sp]);
                    im = dot2_zero(L.im[H][3 * a], v[3 * sp]);
                } else {
                    re = dot2(L.re[H][3 * a + b], v[3 * sp + b], re);
                    im = dot2(L.im[H][3 * a + b], v[3 * sp + b], im);
                }
            }
            acc[3 * sp + a] = make_float2(re, im);
        }
}

// psi + kappa M acc in units of R = max(own scale, M) (a power of two):
// t = acc (kappa M / R) + own (own scale / R), the own halves brought to R in
// FP16 like the neighbours', one rounding per component; then requantise:
// the new record's scale is R 2^e with e the binary exponent of max |t|.
__device__ __forceinline__ float finish_f16s(const float2 acc[12], const half2_t own[12], float so, float M,
                                             float kappa, half2_t q[12]) {
    const float R = fmaxf(so, M);
    const int eR = __builtin_amdgcn_frexp_expf(R);  // R = 2^(eR - 1)
    const _Float16 fo = (_Float16)__builtin_ldexpf(so, 1 - eR);
    const half2_t fo2 = {fo, fo};
    const float kp = kappa * __builtin_ldexpf(M, 1 - eR);
    float2 t[12];
    float m = 0.f;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const half2_t o = own[k] * fo2;
        t[k].x = fma_mix_lo(acc[k].x, kp, o);
        t[k].y = fma_mix_hi(acc[k].y, kp, o);
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) m = max3_abs(t[k].x, t[k].y, m);
    const int et = f16s_exponent(m);
    const float inv = __builtin_ldexpf(1.0f, -et);
#pragma unroll
    for (int k = 0; k < 12; ++k) q[k] = mul_to_half2(t[k].x, t[k].y, inv);
    return m > 0.f ? __builtin_ldexpf(1.0f, eR - 1 + et) : kF16sZeroScale;
}

template <bool BUF>
__device__ __forceinline__ void site_update_f16s(const SmearJob& job, int32_t s, int c0, int c1,
                                                 float kappa) {
    // data: 16-byte chunks (4 half2 each); F16S scales: rows of FP32 after the
    // data, one per record (row 36 + i of the gauge tile, row 12 of a column
    // tile, counted in 4-byte rows)
    const SpatialNeighbours nb = spatial_neighbours(job.g, s);
    const int64_t tbc = tile_bytes(1, 12, QDP_F16S);
    const int64_t cs = tile_site_offset(tbc, 16, s), cs4 = site_off<float>(s, tbc);
    int64_t n16[6], n4[6];
#pragma unroll
    for (int h = 0; h < 6; ++h) {
        const int32_t j = (h & 1) ? nb.bwd[kHopDir[h]] : nb.fwd[kHopDir[h]];
        n16[h] = tile_site_offset(tbc, 16, j);
        n4[h] = site_off<float>(j, tbc);
    }
    F16sLinks L;
    load_links_f16s<BUF>(job.gauge, s, nb, L);

    for (int c = c0; c < c1; ++c) {
        const ChunkRef<BUF> src(job.src[c]);
        const FieldRef<float, BUF> ssc(job.src[c]);
        // Load phase: every neighbour record of this column (6 x 3 chunks and
        // their scales) and the site's own record are requested before any
        // arithmetic, so the wavefront waits for memory once per column.
        half2_t v[6][12], own[12];
        float vsc[6], so;
#pragma unroll
        for (int h = 0; h < 6; ++h) {
            load_elems<0, 12>(src, n16[h], v[h]);
            vsc[h] = ssc.load(12, n4[h]);
        }
        load_elems<0, 12, true>(src, cs, own);  // read once: non-temporal
        so = ssc.load(12, cs4);
        __builtin_amdgcn_sched_barrier(0);

        const F16sHopScale S = hop_scale_f16s(L, vsc);
        float2 acc[12];
        hop_accumulate_f16s<0>(acc, L, S, v[0]);
        hop_accumulate_f16s<1>(acc, L, S, v[1]);
        hop_accumulate_f16s<2>(acc, L, S, v[2]);
        hop_accumulate_f16s<3>(acc, L, S, v[3]);
        hop_accumulate_f16s<4>(acc, L, S, v[4]);
        hop_accumulate_f16s<5>(acc, L, S, v[5]);
        half2_t q[12];
        const float scale = finish_f16s(acc, own, so, S.M, kappa, q);
        store_elems<12, true>(ChunkRef<BUF>(job.dst[c]), cs, q);
        FieldRef<float, BUF>(job.dst[c]).store_stream(scale, 12, cs4);
    }
}

template <int PREC, bool BUF>
__device__ __forceinline__ void site_update(const SmearJob& job, int32_t s, int c0, int c1,
                                            double kappa) {
    if constexpr (PREC == QDP_F64) {
        site_update_real<double, BUF>(job, s, c0, c1, kappa);
    } else if constexpr (PREC == QDP_F32) {
        site_update_real<float, BUF>(job, s, c0, c1, (float)kappa);
    } else {
        site_update_f16s<BUF>(job, s, c0, c1, (float)kappa);
    }
}

// Thread -> (site, column group) for block `tile` of a range of sites.  The
// site_waves wavefronts of a block take consecutive 64-site tiles, or, with
// zstride > 0, tiles zstride apart: blocks p * zstride + r, r < zstride, cover
// the group of site_waves * zstride tiles starting at tile p * site_waves *
// zstride, wave w taking tile p * site_waves * zstride + w * zstride + r.
// `wave` is the wavefront's index among the block's waves of this range.
template <int PREC, bool BUF>
__device__ __forceinline__ void tile_update(const SmearJob& job, int64_t tile, int64_t site_begin,
                                           int64_t site_count, int site_waves, int col_groups, int zstride,
                                           double kappa, int wave) {
    const int lane = threadIdx.x & 63;
    const int group = wave % col_groups, sw = wave / col_groups;
    int64_t t64;
    if (zstride > 0) {
        const int64_t p = tile / zstride, r = tile - p * zstride;
        t64 = (p * site_waves + sw) * zstride + r;
    } else {
        t64 = tile * site_waves + sw;
    }
    const int64_t local = t64 * 64 + lane;
    if (local >= site_count) return;
    const int cpt = (job.ncols + col_groups - 1) / col_groups;
    const int c0 = group * cpt;
    const int c1 = min(job.ncols, c0 + cpt);
    if (c0 >= c1) return;
    site_update<PREC, BUF>(job, (int32_t)(site_begin + local), c0, c1, kappa);
}

// OCC is the occupancy target handed to the register allocator (waves per
// SIMD; 0 = the compiler's choice).  More waves hide more memory latency but
// leave fewer registers for the six links and the prefetched neighbours.
template <int PREC, int OCC, bool BUF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC ? OCC : 1))) void smear_kernel(
    SmearJob job, SmearLaunch ln) {
    int64_t b = blockIdx.x;
    if (ln.xcd == 1) {
        b = xcd_logical_block(b, gridDim.x);
    } else if (ln.xcd == 2) {
        // groups of xcd_group consecutive logical blocks each on one XCD
        // (blocks are dispatched to the XCDs in turn): XCD x takes groups
        // x, x + 8, x + 16, ..., so the eight groups in flight are adjacent
        const int64_t x = b & 7, j = b >> 3;
        b = (x + 8 * (j / ln.xcd_group)) * ln.xcd_group + j % ln.xcd_group;
    }
    if (b >= ln.nlogical) return;
    // the wave index is uniform across the wavefront: keep it (and the
    // column range it selects) in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (ln.interleave == 2) {
        // one block, both parities: even waves take the even tiles, odd
        // waves the odd tiles with the same indices (each other's x, y and,
        // z-stacked, z neighbours, so they meet in the CU's vector cache)
        tile_update<PREC, BUF>(job, b, (wave & 1) * job.g.Vh, job.g.Vh, ln.site_waves / 2, 1, ln.zstride,
                               ln.kappa, wave >> 1);
    } else if (ln.interleave) {
        // the even tile and the odd tile with the same index are each other's
        // neighbours: updating them together lets the L2 serve both
        const int64_t parity = b & 1;
        tile_update<PREC, BUF>(job, b >> 1, parity * job.g.Vh, job.g.Vh, ln.site_waves, ln.col_groups,
                               ln.zstride, ln.kappa, wave);
    } else {
        tile_update<PREC, BUF>(job, b, ln.site_begin, ln.site_count, ln.site_waves, ln.col_groups, ln.zstride,
                               ln.kappa, wave);
    }
}

// ---------------------------------------------------------------------------
// Whole-lattice F16S update with the x/y neighbour window staged in LDS
// ---------------------------------------------------------------------------
// A block of 2 S wavefronts updates the checkerboard index range
// [i0, i0 + 64 S) of both parities (waves 0 .. S-1 the even sites, S .. 2S-1
// the odd ones).  The x and y neighbours of those sites and the sites
// themselves lie in the index window [i0 - Lx/2, i0 + 64 S + Lx/2) of the two
// parities, except where a y hop wraps around the lattice.  Per column the
// block copies that window of both parities into LDS once, with buffer loads
// that write LDS directly (no registers), and every thread reads its own
// record and its x and y neighbours from there instead of fetching each
// record from the vector cache seven times.  The copy of column c + 1 runs
// while column c is computed (two LDS buffers, one barrier per column).  The
// z neighbours come from memory into registers, requested as soon as the
// current column's z terms are done.  Same per-site arithmetic and hop order
// as every other variant, so the same bits.
//
// Block order: block b takes i0 = 64 S b, or, with y bands (ln.bands > 1),
// the lattice's (x, y) planes of a parity are cut into bands of Ly / bands
// rows and the blocks walk band 0 of every plane, then band 1, ...; with the
// XCD-aware mapping each XCD then walks one band over its share of the
// planes, so the z neighbours it reads lie one band-plane, not one plane,
// behind or ahead of the sites it updates, and stay in its L2 until reused.
//
// LDS buffer layout: rows of Wp = 64 (S + 1) slots, window site w of parity
// p in slot w (the slots past the window hold copies of its last site and
// are never read): chunk row r at ((p * 3 + r) * Wp + w) * 16, then the scale
// rows at 96 Wp + (p * Wp + w) * 4.  The window, 64 S + Lx sites, fits a
// row for Lx/2 <= 32.  The two buffers are separate arrays and the column
// loop is unrolled by two, so that every LDS access names its buffer
// statically: the compiler then knows that reading one buffer does not
// depend on the copy in flight into the other and does not wait for it.
constexpr int32_t kLdsMaxHalfX = 32;
__host__ __device__ constexpr int32_t lds_row_slots(int S) { return 64 * (S + 1); }
__host__ __device__ constexpr int64_t lds_buffer_bytes(int S) { return (int64_t)lds_row_slots(S) * 104; }

typedef __attribute__((address_space(3))) void lds_void_t;

// s_waitcnt vmcnt(0): every load of this wave has landed, including the
// copies into LDS (whose completion the compiler does not order with the
// barrier that publishes them to the other waves) and the registers of the
// next column's z records (so the next column starts with nothing in flight
// and its first LDS reads need no wait on the copy issued before them).
__device__ __forceinline__ void vm_wait_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

template <int S>
__global__ __launch_bounds__(128 * S) __attribute__((amdgpu_waves_per_eu(2))) void smear_lds_kernel(
    SmearJob job, SmearLaunch ln) {
    constexpr int32_t Wp = lds_row_slots(S);
    __shared__ __attribute__((aligned(16))) char ldsA[lds_buffer_bytes(S)];
    __shared__ __attribute__((aligned(16))) char ldsB[lds_buffer_bytes(S)];
    const Geometry& g = job.g;
    int64_t b = blockIdx.x;
    if (ln.xcd == 1) b = xcd_logical_block(b, gridDim.x);
    if (b >= ln.nlogical) return;  // whole block: uniform, before any barrier

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int32_t Vh = (int32_t)g.Vh;
    const int32_t q = wave >= S ? 1 : 0;  // parity of this wave's sites
    int32_t i0 = (int32_t)b * 64 * S;
    if (ln.bands > 1) {
        // blocks per band of one plane, then (band, plane, block in band)
        const int32_t plane = g.Lxh * g.L[1], band_sites = plane / ln.bands, per_band = band_sites / (64 * S);
        const int32_t planes = Vh / plane;
        const int32_t bnd = (int32_t)b / (planes * per_band), r = (int32_t)b - bnd * planes * per_band;
        i0 = (r / per_band) * plane + bnd * band_sites + (r % per_band) * 64 * S;
    }
    const int32_t i = i0 + 64 * (wave - q * S) + lane;
    const bool active = i < Vh;
    const int32_t s = q * Vh + (active ? i : Vh - 1);  // a valid site for the inactive lanes' addresses
    const int32_t wbeg = max(0, i0 - g.Lxh);
    const int32_t wlen = min(Vh, i0 + 64 * S + g.Lxh) - wbeg;
    const int64_t tbc = tile_bytes(1, 12, QDP_F16S);

    const SpatialNeighbours nb = spatial_neighbours(g, s);
    const int32_t ob = (1 - q) * Vh;
    // hops 2..5 (y and x) from the window: slot, or -1 when outside it
    int32_t slot[6];
#pragma unroll
    for (int h = 2; h < 6; ++h) {
        const int32_t j = ((h & 1) ? nb.bwd[kHopDir[h]] : nb.fwd[kHopDir[h]]) - ob - wbeg;
        slot[h] = (j >= 0 && j < wlen) ? j : -1;
    }
    const int32_t own_slot = (s - q * Vh) - wbeg;
    int64_t n16[6], n4[6];
#pragma unroll
    for (int h = 0; h < 6; ++h) {
        const int32_t j = (h & 1) ? nb.bwd[kHopDir[h]] : nb.fwd[kHopDir[h]];
        n16[h] = tile_site_offset(tbc, 16, j);
        n4[h] = site_off<float>(j, tbc);
    }
    const int64_t cs = tile_site_offset(tbc, 16, s), cs4 = site_off<float>(s, tbc);
    F16sLinks L;
    load_links_f16s<true>(job.gauge, s, nb, L);

    // copy the window of column c into an LDS buffer: the eight (parity p,
    // row r; r = 3 the scales) rows dealt to the waves in turn, S + 1 full
    // 64-lane pieces each (no lane divergence: lanes past the window copy
    // its last site into padding slots).  The byte offsets of a wave's
    // pieces are the same for every column: computed once.
    constexpr int kRows = 8 / (2 * S);  // rows per wave
    int32_t stage_off[kRows][S + 1];
#pragma unroll
    for (int jj = 0; jj < kRows; ++jj) {
        const int j = wave + 2 * S * jj, p = j >> 2, r = j & 3;
#pragma unroll
        for (int k = 0; k <= S; ++k) {
            const int32_t site = p * Vh + wbeg + min(64 * k + lane, wlen - 1);
            stage_off[jj][k] = (int32_t)(r < 3 ? tile_site_offset(tbc, 16, site) : site_off<float>(site, tbc));
        }
    }
    auto stage = [&](int c, char* base) {
        const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(job.src[c]);
#pragma unroll
        for (int jj = 0; jj < kRows; ++jj) {
            const int j = wave + 2 * S * jj, p = j >> 2, r = j & 3;
#pragma unroll
            for (int k = 0; k <= S; ++k) {
                const int vo = stage_off[jj][k];
                if (r < 3)
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(
                        rs, (lds_void_t*)(base + ((p * 3 + r) * Wp + 64 * k) * 16), 16, vo, r * 1024, 0, 0);
                else
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(
                        rs, (lds_void_t*)(base + 96 * Wp + (p * Wp + 64 * k) * 4), 4, vo, 12 * 256, 0, 0);
            }
        }
    };
    auto lds_record = [&](const char* base, int p, int32_t sl, half2_t v[12]) {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const Chunk<half2_t> ch = __builtin_bit_cast(
                Chunk<half2_t>, *reinterpret_cast<const u32x4_t*>(base + ((p * 3 + r) * Wp + sl) * 16));
#pragma unroll
            for (int j = 0; j < 4; ++j) v[4 * r + j] = ch.v[j];
        }
    };
    auto lds_scale = [&](const char* base, int p, int32_t sl) {
        return *reinterpret_cast<const float*>(base + 96 * Wp + (p * Wp + sl) * 4);
    };

    // A y hop that wraps around the lattice leaves the window: that record
    // (at most one per site for Ly >= 3, none for Ly = 2, x hops never) is
    // fetched from memory with the z neighbours, one column ahead, so that
    // no wait on memory falls between the start of a column and its barrier.
    const int32_t xh = slot[2] < 0 ? 2 : (slot[3] < 0 ? 3 : -1);
    const bool wave_has_x = __builtin_amdgcn_ballot_w64(xh >= 0) != 0;
    const int64_t x16 = xh == 3 ? n16[3] : n16[2], x4 = xh == 3 ? n4[3] : n4[2];

    const int c1 = job.ncols;
    half2_t zv[2][12], xv[12];
    float zsc[2], xsc = 0.f;
    auto load_z = [&](int c) {
        const ChunkRef<true> src(job.src[c]);
        const FieldRef<float, true> ssc(job.src[c]);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            load_elems<0, 12>(src, n16[h], zv[h]);
            zsc[h] = ssc.load(12, n4[h]);
        }
        if (wave_has_x && xh >= 0) {
            load_elems<0, 12>(src, x16, xv);
            xsc = ssc.load(12, x4);
        }
    };
    // column c from buffer rd while column c + 1 is copied into buffer wr
    auto column = [&](int c, const char* rd, char* wr) {
        if (c + 1 < c1) stage(c + 1, wr);
        float nsc[6];
        nsc[0] = zsc[0];
        nsc[1] = zsc[1];
#pragma unroll
        for (int h = 2; h < 6; ++h) nsc[h] = lds_scale(rd, 1 - q, max(slot[h], 0));
        if (wave_has_x) {
            nsc[2] = xh == 2 ? xsc : nsc[2];
            nsc[3] = xh == 3 ? xsc : nsc[3];
        }
        const float so = lds_scale(rd, q, own_slot);
        const F16sHopScale H = hop_scale_f16s(L, nsc);
        float2 acc[12];
        hop_accumulate_f16s<0>(acc, L, H, zv[0]);
        hop_accumulate_f16s<1>(acc, L, H, zv[1]);
        half2_t v[12];
        lds_record(rd, 1 - q, max(slot[2], 0), v);
        if (wave_has_x) {
#pragma unroll
            for (int k = 0; k < 12; ++k) v[k] = xh == 2 ? xv[k] : v[k];
        }
        hop_accumulate_f16s<2>(acc, L, H, v);
        lds_record(rd, 1 - q, max(slot[3], 0), v);
        if (wave_has_x) {
#pragma unroll
            for (int k = 0; k < 12; ++k) v[k] = xh == 3 ? xv[k] : v[k];
        }
        hop_accumulate_f16s<3>(acc, L, H, v);
        // the next column's z (and wrapped y) records: the registers are free
        // now.  Requested on every column (the last one fetches its own again):
        // a conditional load would make the compiler copy these registers
        // around the branch on every column.
        load_z(min(c + 1, c1 - 1));
        lds_record(rd, 1 - q, slot[4], v);
        hop_accumulate_f16s<4>(acc, L, H, v);
        lds_record(rd, 1 - q, slot[5], v);
        hop_accumulate_f16s<5>(acc, L, H, v);
        half2_t own[12], out[12];
        lds_record(rd, q, own_slot, own);
        const float scale = finish_f16s(acc, own, so, H.M, (float)ln.kappa, out);
        if (active) {
            store_elems<12, true>(ChunkRef<true>(job.dst[c]), cs, out);
            FieldRef<float, true>(job.dst[c]).store_stream(scale, 12, cs4);
        }
        vm_wait_all();
        __syncthreads();
    };

    stage(0, ldsA);
    load_z(0);
    vm_wait_all();
    __syncthreads();
    for (int c = 0; c < c1; c += 2) {
        column(c, ldsA, ldsB);
        if (c + 1 < c1) column(c + 1, ldsB, ldsA);
    }
}

// Multi-lattice kernel over a work list of (lattice, tile) items, ordered by
// lattice; a lattice's items alternate between its even and its odd tiles
// (even tile k and odd tile k hold each other's neighbours).  Persistent
// form: a grid of as many blocks as the chip holds at once, block b taking
// items b, b + grid, b + 2 grid, ...; at every step the blocks in flight
// work on one contiguous run of items (one XCD's blocks on one sub-run when
// the mapping is XCD-aware), so neighbouring tiles are read while in L2, as
// in a one-lattice launch.  One-item form (ln.one_item): a block per item,
// the hardware dispatching them in order, so the blocks in flight never
// drift apart over the list.
template <int PREC, int OCC, bool BUF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC ? OCC : 1))) void smear_batch_kernel(
    const SmearJob* __restrict__ jobs, const int64_t* __restrict__ tile_start, int32_t njobs, SmearLaunch ln) {
    const int64_t ntiles = tile_start[njobs];
    int64_t b = blockIdx.x;
    if (ln.xcd) b = xcd_logical_block(b, gridDim.x);
    const int64_t stride = ln.one_item ? ntiles : (int64_t)gridDim.x;
    int j = 0;
    for (int64_t t = b; t < ntiles; t += stride) {
        // the item's lattice: the last j with tile_start[j] <= t
        int lo = j, hi = njobs;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (tile_start[mid] <= t) lo = mid;
            else hi = mid;
        }
        j = lo;
        const SmearJob& job = jobs[j];
        const int64_t u = t - tile_start[j];
        tile_update<PREC, BUF>(job, u >> 1, (u & 1) * job.g.Vh, job.g.Vh, ln.site_waves, ln.col_groups, 0,
                               ln.kappa, __builtin_amdgcn_readfirstlane(threadIdx.x >> 6));
    }
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------

namespace {

struct Launch {
    void* func;
    dim3 grid, block;
    unsigned shmem = 0;      // dynamic LDS bytes
    std::vector<char> args;  // packed argument values
    std::vector<size_t> arg_offsets;
};

template <typename... A>
void pack_args(Launch& L, const A&... a) {
    size_t off = 0;
    auto add = [&](const void* p, size_t n) {
        off = (off + 7) & ~size_t(7);
        L.arg_offsets.push_back(off);
        L.args.resize(off + n);
        std::memcpy(L.args.data() + off, p, n);
        off += n;
    };
    (add(&a, sizeof(A)), ...);
}

std::vector<void*> arg_pointers(Launch& L) {
    std::vector<void*> p;
    for (size_t o : L.arg_offsets) p.push_back(L.args.data() + o);
    return p;
}

// Launch a sequence of kernels in order (from a cached HIP graph when
// use_graph).  Each launch depends on the one before it: the two subset
// passes of an iteration could run concurrently, but measured that way they
// are no faster and each one's duration stops being observable.
qdp_status run_launches(Ctx* ctx, std::vector<Launch>& ls, bool use_graph) {
    if (ls.empty()) return QDP_OK;
    if (!use_graph || ls.size() < 2) {
        for (auto& L : ls) {
            auto p = arg_pointers(L);
            QDP_HIP(ctx, hipLaunchKernel(L.func, L.grid, L.block, p.data(), L.shmem, ctx->stream));
        }
        return QDP_OK;
    }
    // Graph cache keyed by every launch's function, shape and argument bytes.
    std::string key;
    for (auto& L : ls) {
        key.append(reinterpret_cast<const char*>(&L.func), sizeof(L.func));
        key.append(reinterpret_cast<const char*>(&L.grid), sizeof(L.grid));
        key.append(reinterpret_cast<const char*>(&L.block), sizeof(L.block));
        key.append(reinterpret_cast<const char*>(&L.shmem), sizeof(L.shmem));
        key.append(L.args.data(), L.args.size());
    }
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        if (ctx->graphs.size() >= 16) {
            auto victim = ctx->graphs.begin();
            for (auto g = ctx->graphs.begin(); g != ctx->graphs.end(); ++g)
                if (g->second.last_use < victim->second.last_use) victim = g;
            // the least recently used graph may still be running on the stream
            QDP_HIP(ctx, hipStreamSynchronize(ctx->stream));
            hipGraphExecDestroy(victim->second.exec);
            ctx->graphs.erase(victim);
        }
        hipGraph_t graph;
        QDP_HIP(ctx, hipGraphCreate(&graph, 0));
        hipGraphNode_t prev = nullptr;
        for (size_t i = 0; i < ls.size(); ++i) {
            Launch& L = ls[i];
            auto p = arg_pointers(L);
            hipKernelNodeParams np{};
            np.func = L.func;
            np.gridDim = L.grid;
            np.blockDim = L.block;
            np.sharedMemBytes = L.shmem;
            np.kernelParams = p.data();
            np.extra = nullptr;
            hipGraphNode_t node;
            hipError_t e = hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &np);
            if (e != hipSuccess) {
                hipGraphDestroy(graph);
                return hip_error(ctx, e, "hipGraphAddKernelNode");
            }
            prev = node;
        }
        hipGraphExec_t exec;
        hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_error(ctx, e, "hipGraphInstantiate");
        it = ctx->graphs.emplace(key, GraphEntry{exec, 0}).first;
    }
    it->second.last_use = ++ctx->graph_tick;
    QDP_HIP(ctx, hipGraphLaunch(it->second.exec, ctx->stream));
    return QDP_OK;
}

// Kernel variants: occupancy target (FP64 keeps the compiler's choice: its
// links alone need 216 registers) x addressing (buffer / flat).
template <int PREC, bool BUF>
void* smear_func_occ(int occ, bool batch) {
    if constexpr (PREC == QDP_F64) {
        return batch ? reinterpret_cast<void*>(&smear_batch_kernel<PREC, 0, BUF>)
                     : reinterpret_cast<void*>(&smear_kernel<PREC, 0, BUF>);
    } else {
        if (batch)
            return occ == 3 ? reinterpret_cast<void*>(&smear_batch_kernel<PREC, 3, BUF>)
                 : occ == 2 ? reinterpret_cast<void*>(&smear_batch_kernel<PREC, 2, BUF>)
                            : reinterpret_cast<void*>(&smear_batch_kernel<PREC, 0, BUF>);
        return occ == 3 ? reinterpret_cast<void*>(&smear_kernel<PREC, 3, BUF>)
             : occ == 2 ? reinterpret_cast<void*>(&smear_kernel<PREC, 2, BUF>)
                        : reinterpret_cast<void*>(&smear_kernel<PREC, 0, BUF>);
    }
}

template <bool BUF>
void* smear_func_buf(int prec, int occ, bool batch) {
    switch (prec) {
        case QDP_F64: return smear_func_occ<QDP_F64, BUF>(occ, batch);
        case QDP_F32: return smear_func_occ<QDP_F32, BUF>(occ, batch);
        default: return smear_func_occ<QDP_F16S, BUF>(occ, batch);
    }
}

void* smear_func(int prec, const qdp_launch_shape& sh, bool batch) {
    return sh.flat ? smear_func_buf<false>(prec, sh.waves_per_simd, batch)
                   : smear_func_buf<true>(prec, sh.waves_per_simd, batch);
}

// Whether the LDS-window kernel runs this launch: F16S, the whole lattice,
// buffer addressing, and a window that fits its LDS rows (Lx <= 64).
bool lds_eligible(int prec, const SmearJob& job, int64_t begin, int64_t count, const qdp_launch_shape& sh) {
    if (sh.lds < 1 || sh.lds > 2 || prec != QDP_F16S || sh.flat || begin != 0 || count != job.g.V) return false;
    return job.g.Lxh <= kLdsMaxHalfX;
}

// y bands of the LDS-window kernel for zstack = 1 (two, or three when two
// do not fit) or 2 (four), when Ly splits evenly and a band of one plane is
// a whole number of blocks; else 1 (plain order).
int32_t lds_bands(const SmearJob& job, const qdp_launch_shape& sh) {
    auto fits = [&](int32_t bands) {
        return job.g.L[1] % bands == 0 && ((int64_t)job.g.Lxh * job.g.L[1] / bands) % (64LL * sh.lds) == 0;
    };
    if (sh.zstack == 1) {  // the fewest bands that fit: 2, else 3
        if (fits(2)) return 2;
        if (fits(3)) return 3;
    }
    if (sh.zstack == 2 && fits(4)) return 4;
    return 1;
}

// A pass over [begin, begin + count); count == V (the whole lattice) runs
// the two parities' tiles interleaved.
Launch make_single_launch(int prec, const SmearJob& job, int64_t begin, int64_t count,
                          const qdp_launch_shape& sh, double kappa) {
    if (lds_eligible(prec, job, begin, count, sh)) {
        SmearLaunch ln{};
        ln.site_begin = 0;
        ln.site_count = job.g.V;
        ln.interleave = 1;
        ln.xcd = sh.xcd ? 1 : 0;
        ln.kappa = kappa;
        ln.bands = lds_bands(job, sh);
        ln.nlogical = (job.g.Vh + 64LL * sh.lds - 1) / (64LL * sh.lds);
        const int64_t grid = ln.xcd ? (ln.nlogical + 7) / 8 * 8 : ln.nlogical;
        Launch L;
        L.func = sh.lds == 1 ? reinterpret_cast<void*>(&smear_lds_kernel<1>)
                             : reinterpret_cast<void*>(&smear_lds_kernel<2>);
        L.grid = dim3((unsigned)grid);
        L.block = dim3((unsigned)(128 * sh.lds));
        pack_args(L, job, ln);
        return L;
    }
    SmearLaunch ln{};
    ln.site_begin = begin;
    ln.site_count = count;
    ln.interleave = (begin == 0 && count == job.g.V) ? 1 : 0;
    // zstack = 2 on the whole lattice: both parities in one block (half of
    // the waves each), single column group
    const bool mixed = ln.interleave && sh.zstack == 2 && sh.col_groups == 1 && sh.site_waves % 2 == 0;
    if (mixed) ln.interleave = 2;
    const int per_parity_waves = mixed ? sh.site_waves / 2 : sh.site_waves;
    // z-stacked blocks: one (x, y) plane of a parity, Lx/2 * Ly sites, in
    // 64-site tiles (rounded)
    ln.zstride = (sh.zstack && per_parity_waves > 1)
                     ? (int32_t)std::max<int64_t>(1, ((int64_t)job.g.Lxh * job.g.L[1] + 32) / 64) : 0;
    const int64_t range = ln.interleave ? job.g.Vh : count;  // sites of one parity's range
    int64_t blocks;
    if (ln.zstride > 0) {
        const int64_t group = (int64_t)per_parity_waves * ln.zstride;
        blocks = ((range + 63) / 64 + group - 1) / group * ln.zstride;
    } else {
        blocks = (range + 64LL * per_parity_waves - 1) / (64LL * per_parity_waves);
    }
    ln.nlogical = ln.interleave == 1 ? 2 * blocks : blocks;
    ln.site_waves = sh.site_waves;
    ln.col_groups = sh.col_groups;
    ln.xcd = sh.xcd;
    ln.kappa = kappa;
    int64_t grid = ln.nlogical;
    if (sh.xcd == 1) {
        grid = (grid + 7) / 8 * 8;
    } else if (sh.xcd == 2) {
        // a group: the blocks of one z-stack group (both parities' in the
        // interleaved launch), or 8 blocks without z-stacking
        ln.xcd_group = ln.zstride > 0 ? (ln.interleave == 1 ? 2 : 1) * ln.zstride : 8;
        const int64_t unit = 8LL * ln.xcd_group;
        grid = (grid + unit - 1) / unit * unit;
    }
    Launch L;
    L.func = smear_func(prec, sh, false);
    L.grid = dim3((unsigned)grid);
    L.block = dim3((unsigned)(64 * sh.site_waves * sh.col_groups));
    pack_args(L, job, ln);
    return L;
}

qdp_launch_shape default_shape() { return qdp_launch_shape{4, 1, 1, 2, 0, 0, 0}; }

// A candidate launch shape replaces the best one so far only when it is
// faster by more than 0.5 %.
constexpr float kTuneMargin = 0.995f;

// Validate a list of columns against the gauge field; returns precision and
// lattice through the out arguments.
qdp_status check_columns(Ctx* ctx, uint64_t gauge, const uint64_t* cols, int32_t ncols,
                         uint64_t* lattice, int32_t* prec) {
    Field* gf = find_field(ctx, gauge);
    if (!gf) return set_error(ctx, QDP_ERR_STATE, "smear: unknown gauge handle");
    if (gf->type != QDP_GAUGE) return set_error(ctx, QDP_ERR_TYPE, "smear: links must be a GAUGE field");
    for (int32_t c = 0; c < ncols; ++c) {
        Field* f = find_field(ctx, cols[c]);
        if (!f) return set_error(ctx, QDP_ERR_STATE, "smear: unknown column handle");
        if (f->type != QDP_FERMION) return set_error(ctx, QDP_ERR_TYPE, "smear: columns must be FERMION fields");
        if (f->lattice != gf->lattice) return set_error(ctx, QDP_ERR_LATTICE, "smear: column on another lattice");
        if (f->prec != gf->prec)
            return set_error(ctx, QDP_ERR_UNSUPPORTED, "smear: column precision differs from the links'");
    }
    *lattice = gf->lattice;
    *prec = gf->prec;
    return QDP_OK;
}

qdp_status check_aliasing(Ctx* ctx, const uint64_t* src, const uint64_t* dst, int32_t ncols) {
    for (int32_t a = 0; a < ncols; ++a)
        for (int32_t b = 0; b < ncols; ++b) {
            if (a == b) continue;
            if (dst[a] == dst[b] || dst[a] == src[b])
                return set_error(ctx, QDP_ERR_ALIAS, "smear: destination column %d aliases column %d", a, b);
        }
    return QDP_OK;
}

// Buffer addressing needs every byte offset of the links and of a column
// below 4 GiB (and is off in a context made with QDP_INIT_FLAT_ADDRESSING).
bool needs_flat(Ctx* ctx, uint64_t gauge, uint64_t lattice, int32_t prec) {
    if (ctx->flags & QDP_INIT_FLAT_ADDRESSING) return true;
    const Geometry& g = find_lattice(ctx, lattice)->geo;
    const int64_t limit = (int64_t(1) << 32) - 1;
    return find_field(ctx, gauge)->bytes > limit || field_bytes(g, QDP_FERMION, prec) > limit;
}

// Time one launch shape on the first pass (it writes only the buffer the
// first real iteration overwrites).
qdp_status time_shape(Ctx* ctx, int prec, const SmearJob& job, int64_t begin, int64_t count,
                      const qdp_launch_shape& sh, double kappa, float* ms) {
    Launch L = make_single_launch(prec, job, begin, count, sh, kappa);
    auto p = arg_pointers(L);
    hipEvent_t e0, e1;
    QDP_HIP(ctx, hipEventCreate(&e0));
    QDP_HIP(ctx, hipEventCreate(&e1));
    float best = 1e30f;
    for (int rep = 0; rep < 5; ++rep) {
        hipEventRecord(e0, ctx->stream);
        hipLaunchKernel(L.func, L.grid, L.block, p.data(), L.shmem, ctx->stream);
        hipEventRecord(e1, ctx->stream);
        hipError_t err = hipEventSynchronize(e1);
        if (err != hipSuccess) {
            hipEventDestroy(e0);
            hipEventDestroy(e1);
            return hip_error(ctx, err, "autotune launch");
        }
        float t = 0.f;
        hipEventElapsedTime(&t, e0, e1);
        if (rep > 0) best = std::min(best, t);
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    *ms = best;
    return QDP_OK;
}

qdp_status choose_shape(Ctx* ctx, const SmearTuneKey& key, int prec, const SmearJob& job,
                        int64_t begin, int64_t count, double kappa, int flat, qdp_launch_shape* out) {
    if (ctx->forced.site_waves > 0) {
        *out = ctx->forced;
        out->flat = out->flat | flat;
        return QDP_OK;
    }
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end()) {
        *out = it->second;
        return QDP_OK;
    }
    qdp_launch_shape best = default_shape();
    best.flat = flat;
    const bool log = std::getenv("QDP_AUTOTUNE_LOG") != nullptr;
    const int64_t work = count * job.ncols;
    if (!(ctx->flags & QDP_INIT_NO_AUTOTUNE) && work >= (1 << 20)) {
        std::vector<qdp_launch_shape> cands;
        const int groups[] = {1, 2, 3, 4, 6};
        for (int sw : {1, 2, 4})
            for (int cg : groups) {
                if (sw * cg > 4 || cg > job.ncols) continue;
                for (int xcd : {0, 1, 2})
                    for (int occ : {0, 2, 3})
                        for (int zs : {0, 1, 2}) {
                            if ((prec == QDP_F64 && occ) || (zs && sw == 1) || (xcd == 2 && !zs)) continue;
                            if (zs == 2 && (count != job.g.V || cg != 1 || sw % 2)) continue;
                            cands.push_back(qdp_launch_shape{sw, cg, xcd, occ, flat, zs, 0});
                        }
            }
        // two-wave rows (S = 2) and the banded orders first: they fetch
        // fewer bytes, so on a tie within the timing margin the one that
        // loads the memory system less is kept (over whole smearing runs it
        // is also the faster one)
        for (int S : {2, 1})
            for (int xcd : {0, 1})
                for (int zs : {1, 2, 0}) {
                    const qdp_launch_shape sh{1, 1, xcd, 0, flat, zs, S};
                    if (lds_eligible(prec, job, begin, count, sh) && (zs == 0 || lds_bands(job, sh) > 1))
                        cands.push_back(sh);
                }
        // two rounds over the candidates, each keeping its faster time, so
        // that no candidate's figure depends on where in the sequence the
        // clocks or caches happened to be
        std::vector<float> t(cands.size(), 1e30f);
        for (int round = 0; round < 2; ++round)
            for (size_t i = 0; i < cands.size(); ++i) {
                float ms;
                QDP_CHECK(time_shape(ctx, prec, job, begin, count, cands[i], kappa, &ms));
                t[i] = std::min(t[i], ms);
            }
        float best_ms = 1e30f;
        for (size_t i = 0; i < cands.size(); ++i) {
            const qdp_launch_shape& sh = cands[i];
            if (log)
                std::fprintf(stderr, "[qdpmi autotune] prec %d cols %d sites %lld shape %d %d %d %d %d %d %d: %.4f ms\n",
                             prec, job.ncols, (long long)count, sh.site_waves, sh.col_groups, sh.xcd,
                             sh.waves_per_simd, sh.flat, sh.zstack, sh.lds, t[i]);
            // a later candidate must win by more than the timing noise:
            // equal kernels (the occupancy targets often compile to the same
            // code) keep the first, so the choice repeats run to run
            if (t[i] < best_ms * kTuneMargin) {
                best_ms = t[i];
                best = sh;
            }
        }
    }
    ctx->tuned[key] = best;
    *out = best;
    return QDP_OK;
}

}  // namespace

void release_graphs(Ctx* ctx) {
    for (auto& kv : ctx->graphs) hipGraphExecDestroy(kv.second.exec);
    ctx->graphs.clear();
}

qdp_status smear_jacobi_impl(Ctx* ctx, uint64_t gauge, const uint64_t* src, const uint64_t* dst,
                             int32_t ncols, double kappa, int32_t n_iter, int32_t j_decay,
                             int32_t mode) {
    if (ncols < 1 || ncols > 12) return set_error(ctx, QDP_ERR_ARG, "smear: 1..12 columns");
    if (n_iter < 0) return set_error(ctx, QDP_ERR_ARG, "smear: negative iteration count");
    if (!std::isfinite(kappa)) return set_error(ctx, QDP_ERR_ARG, "smear: kappa not finite");
    if (j_decay != 3) return set_error(ctx, QDP_ERR_UNSUPPORTED, "smear: only j_decay = 3 (time)");
    if (mode != QDP_SMEAR_FULL && mode != QDP_SMEAR_EVEN_ODD)
        return set_error(ctx, QDP_ERR_ARG, "smear: unknown mode %d", mode);
    uint64_t lat;
    int32_t prec;
    QDP_CHECK(check_columns(ctx, gauge, src, ncols, &lat, &prec));
    QDP_CHECK(check_columns(ctx, gauge, dst, ncols, &lat, &prec));
    QDP_CHECK(check_aliasing(ctx, src, dst, ncols));
    const Geometry g = find_lattice(ctx, lat)->geo;

    if (n_iter == 0) {
        for (int32_t c = 0; c < ncols; ++c) {
            if (src[c] == dst[c]) continue;
            PinSet pins(ctx);
            char *ps, *pd;
            QDP_CHECK(pins.add(src[c], true, &ps));
            QDP_CHECK(pins.add(dst[c], false, &pd));
            QDP_HIP(ctx, hipMemcpyAsync(pd, ps, find_field(ctx, dst[c])->bytes, hipMemcpyDeviceToDevice,
                                        ctx->stream));
        }
        return QDP_OK;
    }

    // Ping-pong partners: iteration k writes tmp for odd k and dst for even
    // k; with an odd count the result lands in tmp and the storages of tmp
    // and dst are exchanged afterwards.
    std::vector<uint64_t> tmp(ncols, 0);
    struct TmpGuard {
        Ctx* ctx;
        std::vector<uint64_t>* ids;
        ~TmpGuard() {
            for (uint64_t id : *ids)
                if (id) field_destroy(ctx, id);
        }
    } guard{ctx, &tmp};
    for (int32_t c = 0; c < ncols; ++c) QDP_CHECK(field_create(ctx, lat, QDP_FERMION, prec, &tmp[c]));

    {
        PinSet pins(ctx);
        char* pg;
        QDP_CHECK(pins.add(gauge, true, &pg));
        std::vector<char*> ps(ncols), pd(ncols), pt(ncols);
        for (int32_t c = 0; c < ncols; ++c) {
            QDP_CHECK(pins.add(src[c], true, &ps[c]));
            if (dst[c] != src[c]) QDP_CHECK(pins.add(dst[c], false, &pd[c]));
            else pd[c] = ps[c];
            QDP_CHECK(pins.add(tmp[c], false, &pt[c]));
        }

        SmearJob first{}, to_dst{}, to_tmp{};
        first.g = to_dst.g = to_tmp.g = g;
        first.gauge = to_dst.gauge = to_tmp.gauge = pg;
        first.ncols = to_dst.ncols = to_tmp.ncols = ncols;
        for (int32_t c = 0; c < ncols; ++c) {
            first.src[c] = ps[c];
            first.dst[c] = pt[c];
            to_dst.src[c] = pt[c];
            to_dst.dst[c] = pd[c];
            to_tmp.src[c] = pd[c];
            to_tmp.dst[c] = pt[c];
        }

        struct Pass {
            int64_t begin, count;
        };
        std::vector<Pass> passes;
        if (mode == QDP_SMEAR_FULL) passes.push_back({0, g.V});
        else {
            passes.push_back({0, g.Vh});
            passes.push_back({g.Vh, g.Vh});
        }

        SmearTuneKey key{{g.L[0], g.L[1], g.L[2], g.L[3]}, ncols, prec, mode, 0};
        qdp_launch_shape sh;
        const int flat = needs_flat(ctx, gauge, lat, prec) ? 1 : 0;
        QDP_CHECK(choose_shape(ctx, key, prec, first, passes[0].begin, passes[0].count, kappa, flat, &sh));
        ctx->last_shape = sh;

        std::vector<Launch> ls;
        for (int32_t k = 1; k <= n_iter; ++k) {
            const SmearJob& job = k == 1 ? first : (k % 2 == 0 ? to_dst : to_tmp);
            for (const Pass& p : passes) ls.push_back(make_single_launch(prec, job, p.begin, p.count, sh, kappa));
        }
        QDP_CHECK(run_launches(ctx, ls, !(ctx->flags & QDP_INIT_NO_GRAPH)));
        QDP_CHECK(check_launch(ctx, "smear kernel"));
    }
    if (n_iter % 2 == 1) {
        for (int32_t c = 0; c < ncols; ++c)
            if (ctx->cache.swap_storage(dst[c], tmp[c]) != QDP_OK)
                return set_error(ctx, QDP_ERR_STATE, "smear: result hand-over failed");
    }
    return QDP_OK;
}

qdp_status smear_batch_impl(Ctx* ctx, const qdp_smear_job* jobs, int32_t njobs, double kappa,
                            int32_t n_iter) {
    if (n_iter < 0) return set_error(ctx, QDP_ERR_ARG, "smear batch: negative iteration count");
    if (!std::isfinite(kappa)) return set_error(ctx, QDP_ERR_ARG, "smear batch: kappa not finite");
    int32_t prec = -1;
    std::vector<std::vector<uint64_t>> src(njobs), dst(njobs);
    std::vector<uint64_t> lats(njobs);
    for (int32_t j = 0; j < njobs; ++j) {
        const qdp_smear_job& J = jobs[j];
        if (!J.src || !J.dst || J.ncols < 1 || J.ncols > 12)
            return set_error(ctx, QDP_ERR_ARG, "smear batch: job %d needs 1..12 columns", j);
        src[j].assign(J.src, J.src + J.ncols);
        dst[j].assign(J.dst, J.dst + J.ncols);
        int32_t p;
        QDP_CHECK(check_columns(ctx, J.gauge, src[j].data(), J.ncols, &lats[j], &p));
        QDP_CHECK(check_columns(ctx, J.gauge, dst[j].data(), J.ncols, &lats[j], &p));
        QDP_CHECK(check_aliasing(ctx, src[j].data(), dst[j].data(), J.ncols));
        if (prec >= 0 && p != prec)
            return set_error(ctx, QDP_ERR_UNSUPPORTED, "smear batch: all jobs must share one precision");
        prec = p;
    }
    for (int32_t a = 0; a < njobs; ++a)
        for (int32_t b = a + 1; b < njobs; ++b)
            for (uint64_t x : dst[a])
                for (int32_t c = 0; c < jobs[b].ncols; ++c)
                    if (x == dst[b][c] || x == src[b][c])
                        return set_error(ctx, QDP_ERR_ALIAS, "smear batch: jobs %d and %d share a field", a, b);
    if (n_iter == 0) {
        for (int32_t j = 0; j < njobs; ++j)
            QDP_CHECK(smear_jacobi_impl(ctx, jobs[j].gauge, src[j].data(), dst[j].data(), jobs[j].ncols,
                                        kappa, 0, 3, QDP_SMEAR_FULL));
        return QDP_OK;
    }

    std::vector<std::vector<uint64_t>> tmp(njobs);
    struct TmpGuard {
        Ctx* ctx;
        std::vector<std::vector<uint64_t>>* ids;
        ~TmpGuard() {
            for (auto& v : *ids)
                for (uint64_t id : v)
                    if (id) field_destroy(ctx, id);
        }
    } guard{ctx, &tmp};
    for (int32_t j = 0; j < njobs; ++j) {
        tmp[j].assign(jobs[j].ncols, 0);
        for (int32_t c = 0; c < jobs[j].ncols; ++c)
            QDP_CHECK(field_create(ctx, lats[j], QDP_FERMION, prec, &tmp[j][c]));
    }

    int flat = 0;
    std::string tune_key(reinterpret_cast<const char*>(&prec), sizeof prec);
    for (int32_t j = 0; j < njobs; ++j) {
        if (needs_flat(ctx, jobs[j].gauge, lats[j], prec)) flat = 1;
        const Geometry& g = find_lattice(ctx, lats[j])->geo;
        tune_key.append(reinterpret_cast<const char*>(g.L), sizeof g.L);
        tune_key.append(reinterpret_cast<const char*>(&jobs[j].ncols), sizeof(int32_t));
    }

    // work lists for the tile sizes 64 * site_waves, site_waves = 1..4
    PinSet pins(ctx);
    std::vector<SmearJob> h_first(njobs), h_dst(njobs), h_tmp(njobs);
    std::vector<int64_t> h_tiles(4 * (njobs + 1), 0);
    for (int32_t j = 0; j < njobs; ++j) {
        const Geometry& g = find_lattice(ctx, lats[j])->geo;
        char* pg;
        QDP_CHECK(pins.add(jobs[j].gauge, true, &pg));
        SmearJob a{}, b{}, c{};
        a.g = b.g = c.g = g;
        a.gauge = b.gauge = c.gauge = pg;
        a.ncols = b.ncols = c.ncols = jobs[j].ncols;
        for (int32_t k = 0; k < jobs[j].ncols; ++k) {
            char *ps, *pd, *pt;
            QDP_CHECK(pins.add(src[j][k], true, &ps));
            if (dst[j][k] != src[j][k]) QDP_CHECK(pins.add(dst[j][k], false, &pd));
            else pd = ps;
            QDP_CHECK(pins.add(tmp[j][k], false, &pt));
            a.src[k] = ps;
            a.dst[k] = pt;
            b.src[k] = pt;
            b.dst[k] = pd;
            c.src[k] = pd;
            c.dst[k] = pt;
        }
        h_first[j] = a;
        h_dst[j] = b;
        h_tmp[j] = c;
        for (int k = 0; k < 4; ++k) {  // an even and an odd tile per index
            const int64_t tile_sites = 64LL * (k + 1);
            h_tiles[k * (njobs + 1) + j + 1] = h_tiles[k * (njobs + 1) + j] + 2 * ((g.Vh + tile_sites - 1) / tile_sites);
        }
    }
    const size_t jb = sizeof(SmearJob) * njobs;
    const size_t tb = sizeof(int64_t) * 4 * (njobs + 1);
    PoolTemp dev;
    QDP_CHECK(dev.alloc(ctx, (int64_t)(3 * jb + tb + 1024)));
    char* d_first = dev.ptr();
    char* d_dst = d_first + ((jb + 255) & ~size_t(255));
    char* d_tmp = d_dst + ((jb + 255) & ~size_t(255));
    char* d_tiles = d_tmp + ((jb + 255) & ~size_t(255));
    QDP_HIP(ctx, hipMemcpyAsync(d_first, h_first.data(), jb, hipMemcpyHostToDevice, ctx->stream));
    QDP_HIP(ctx, hipMemcpyAsync(d_dst, h_dst.data(), jb, hipMemcpyHostToDevice, ctx->stream));
    QDP_HIP(ctx, hipMemcpyAsync(d_tmp, h_tmp.data(), jb, hipMemcpyHostToDevice, ctx->stream));
    QDP_HIP(ctx, hipMemcpyAsync(d_tiles, h_tiles.data(), tb, hipMemcpyHostToDevice, ctx->stream));

    // one persistent launch over every lattice's tiles with job list J
    auto batch_launch = [&](const char* J, const qdp_launch_shape& sh) {
        const int k = sh.site_waves - 1;  // 1..4, checked by qdp_smear_set_shape
        SmearLaunch ln{};
        ln.site_waves = sh.site_waves;
        ln.col_groups = sh.col_groups;
        ln.xcd = sh.xcd;
        ln.kappa = kappa;
        const int64_t ntiles = h_tiles[k * (njobs + 1) + njobs];
        ln.one_item = sh.zstack == 1 ? 1 : 0;
        Launch L;
        L.func = smear_func(prec, sh, true);
        L.block = dim3((unsigned)(64 * sh.site_waves * sh.col_groups));
        // persistent: as many blocks as are resident at once; one item per
        // block: every item (a multiple of 8 for the XCD mapping either way)
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, L.func, (int)L.block.x, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        int64_t grid = ln.one_item ? ntiles : std::min<int64_t>(ntiles, (int64_t)ctx->num_cus * per_cu);
        grid = std::max<int64_t>(8, (grid + 7) / 8 * 8);
        const int64_t* T = reinterpret_cast<const int64_t*>(d_tiles) + k * (njobs + 1);
        L.grid = dim3((unsigned)grid);
        pack_args(L, reinterpret_cast<const SmearJob*>(J), T, njobs, ln);
        return L;
    };

    qdp_launch_shape sh;
    if (ctx->forced.site_waves > 0) {
        sh = ctx->forced;
        sh.flat |= flat;
    } else if (ctx->tuned_batch.count(tune_key)) {
        sh = ctx->tuned_batch[tune_key];
    } else {
        // time one launch per candidate shape (the first iteration's job list:
        // it writes only the temporaries, which the real iterations overwrite)
        sh = default_shape();
        sh.flat = flat;
        const bool log = std::getenv("QDP_AUTOTUNE_LOG") != nullptr;
        if (!(ctx->flags & QDP_INIT_NO_AUTOTUNE)) {
            float best_ms = 1e30f;
            hipEvent_t e0, e1;
            QDP_HIP(ctx, hipEventCreate(&e0));
            QDP_HIP(ctx, hipEventCreate(&e1));
            const int groups[] = {1, 2, 3, 4, 6};
            for (int one : {0, 1})
            for (int sw : {1, 2, 4})
                for (int cg : groups)
                    for (int xcd : {0, 1})
                        for (int occ : {0, 2, 3}) {
                            if (sw * cg > 4 || (prec == QDP_F64 && occ)) continue;
                            const qdp_launch_shape cand{sw, cg, xcd, occ, flat, one, 0};
                            Launch L = batch_launch(d_first, cand);
                            auto p = arg_pointers(L);
                            float best = 1e30f;
                            for (int rep = 0; rep < 2; ++rep) {
                                hipEventRecord(e0, ctx->stream);
                                hipLaunchKernel(L.func, L.grid, L.block, p.data(), 0, ctx->stream);
                                hipEventRecord(e1, ctx->stream);
                                hipError_t err = hipEventSynchronize(e1);
                                if (err != hipSuccess) {
                                    hipEventDestroy(e0);
                                    hipEventDestroy(e1);
                                    return hip_error(ctx, err, "batch autotune launch");
                                }
                                float t = 0.f;
                                hipEventElapsedTime(&t, e0, e1);
                                if (rep > 0) best = std::min(best, t);
                            }
                            if (log)
                                std::fprintf(stderr, "[qdpmi autotune] batch of %d prec %d shape %d %d %d %d %d %d: %.4f ms\n",
                                             njobs, prec, sw, cg, xcd, occ, flat, one, best);
                            if (best < best_ms * kTuneMargin) {
                                best_ms = best;
                                sh = cand;
                            }
                        }
            hipEventDestroy(e0);
            hipEventDestroy(e1);
        }
        ctx->tuned_batch[tune_key] = sh;
    }
    ctx->last_shape = sh;

    std::vector<Launch> ls;
    for (int32_t k = 1; k <= n_iter; ++k)
        ls.push_back(batch_launch(k == 1 ? d_first : (k % 2 == 0 ? d_dst : d_tmp), sh));
    QDP_CHECK(run_launches(ctx, ls, !(ctx->flags & QDP_INIT_NO_GRAPH)));
    QDP_CHECK(check_launch(ctx, "smear batch kernel"));
    if (n_iter % 2 == 1) {
        for (int32_t j = 0; j < njobs; ++j)
            for (int32_t c = 0; c < jobs[j].ncols; ++c)
                if (ctx->cache.swap_storage(dst[j][c], tmp[j][c]) != QDP_OK)
                    return set_error(ctx, QDP_ERR_STATE, "smear batch: result hand-over failed");
    }
    return QDP_OK;
}

}  // namespace qdpmi
