// Synthetic inputs generated on the device (qdp_fill_random, qdp_fill_point):
// Haar SU(3) gauge links, Gaussian propagator columns and point sources for
// the benchmark and the full-size tests, where generating gigabytes on the
// host would dominate the run.
//
// Counter-based generator: Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
// SC'11).  Complex normal number e of stream sid under key `seed` is the
// Box-Muller transform of two 53-bit uniforms made from the output block of
// counter (e mod 2^32, e div 2^32, sid, 0).  SU(3): Gram-Schmidt (two
// projection passes) on the columns of a 3x3 complex Gaussian, then division
// by the principal cube root of the determinant.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device.hpp"
#include "internal.hpp"

namespace qdpmi {

namespace {

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        const uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
        const uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

__device__ __forceinline__ double uniform53(uint32_t hi, uint32_t lo) {
    const uint64_t k = ((uint64_t)(hi >> 5) << 26) | (uint64_t)(lo >> 6);
    return ((double)k + 0.5) * 0x1p-53;
}

__device__ __forceinline__ double2 complex_normal(uint64_t seed, uint32_t stream, uint64_t e) {
    const uint4 w = philox4x32_10(make_uint4((uint32_t)e, (uint32_t)(e >> 32), stream, 0u), (uint32_t)seed,
                                  (uint32_t)(seed >> 32));
    const double u1 = uniform53(w.x, w.y);
    const double u2 = uniform53(w.z, w.w);
    const double r = sqrt(-2.0 * log(u1));
    const double th = (2.0 * 3.141592653589793) * u2;
    return make_double2(r * cos(th), r * sin(th));
}

// Store one record of n complex doubles at checkerboard site s.
__device__ void store_record(char* base, int32_t prec, int32_t nrec, int32_t ncomp, int32_t rec, int32_t s,
                             const double2* v, int n) {
    if (prec == QDP_F64) {
        for (int k = 0; k < n; ++k) *reinterpret_cast<double2*>(base + comp_offset(nrec, ncomp, prec, rec, k, s)) = v[k];
    } else if (prec == QDP_F32) {
        for (int k = 0; k < n; ++k)
            *reinterpret_cast<float2*>(base + comp_offset(nrec, ncomp, prec, rec, k, s)) =
                make_float2((float)v[k].x, (float)v[k].y);
    } else {
        float m = 0.f;
        for (int k = 0; k < n; ++k) m = fmaxf(m, fmaxf(fabsf((float)v[k].x), fabsf((float)v[k].y)));
        const int e = f16s_exponent(m);
        for (int k = 0; k < n; ++k)
            *reinterpret_cast<half2_t*>(base + comp_offset(nrec, ncomp, prec, rec, k, s)) =
                f16s_encode((float)v[k].x, (float)v[k].y, e);
        *reinterpret_cast<float*>(base + scale_offset(nrec, ncomp, rec, s)) = f16s_scale(m, e);
    }
}

__device__ __forceinline__ double2 cm(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ __launch_bounds__(256) void su3_kernel(Geometry g, char* base, int32_t prec, uint64_t seed) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 4 * g.V) return;
    const int32_t mu = (int32_t)(idx / g.V);
    const int64_t s = idx - mu * g.V;  // lexicographic site
    double2 z[3][3];  // z[row][col]
    for (int k = 0; k < 9; ++k) z[k / 3][k % 3] = complex_normal(seed, 1u, (uint64_t)idx * 9 + k);
    double2 q[3][3];
    for (int j = 0; j < 3; ++j) {
        double2 v[3] = {z[0][j], z[1][j], z[2][j]};
        for (int pass = 0; pass < 2; ++pass)
            for (int k = 0; k < j; ++k) {
                double2 proj = make_double2(0.0, 0.0);
                for (int i = 0; i < 3; ++i) {
                    const double2 t = cm(make_double2(q[i][k].x, -q[i][k].y), v[i]);
                    proj.x += t.x;
                    proj.y += t.y;
                }
                for (int i = 0; i < 3; ++i) {
                    const double2 t = cm(proj, q[i][k]);
                    v[i].x -= t.x;
                    v[i].y -= t.y;
                }
            }
        double nn = 0.0;
        for (int i = 0; i < 3; ++i) nn += v[i].x * v[i].x + v[i].y * v[i].y;
        const double nrm = sqrt(nn);
        for (int i = 0; i < 3; ++i) q[i][j] = make_double2(v[i].x / nrm, v[i].y / nrm);
    }
    // det by cofactor expansion along the first row
    const double2 m0 = cm(q[1][1], q[2][2]), m0b = cm(q[1][2], q[2][1]);
    const double2 m1 = cm(q[1][0], q[2][2]), m1b = cm(q[1][2], q[2][0]);
    const double2 m2 = cm(q[1][0], q[2][1]), m2b = cm(q[1][1], q[2][0]);
    const double2 c0 = cm(q[0][0], make_double2(m0.x - m0b.x, m0.y - m0b.y));
    const double2 c1 = cm(q[0][1], make_double2(m1.x - m1b.x, m1.y - m1b.y));
    const double2 c2 = cm(q[0][2], make_double2(m2.x - m2b.x, m2.y - m2b.y));
    const double2 det = make_double2(c0.x - c1.x + c2.x, c0.y - c1.y + c2.y);
    const double ph = atan2(det.y, det.x);
    const double2 fix = make_double2(cos(-ph / 3.0), sin(-ph / 3.0));
    double2 out[9];
    for (int k = 0; k < 9; ++k) out[k] = cm(q[k / 3][k % 3], fix);
    int32_t c[4];
    int64_t r = s;
    for (int d = 0; d < 4; ++d) {
        c[d] = (int32_t)(r % g.L[d]);
        r /= g.L[d];
    }
    const int32_t cb = (int32_t)cb_index(g, c[0], c[1], c[2], c[3]);
    store_record(base, prec, 4, 9, mu, cb, out, 9);
}

__global__ __launch_bounds__(256) void gaussian_kernel(Geometry g, char* base, int32_t prec, uint64_t seed,
                                                       int32_t column, double scale) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    double2 v[12];
    for (int k = 0; k < 12; ++k) {
        const double2 z = complex_normal(seed, 2u, ((uint64_t)column * g.V + s) * 12 + k);
        v[k] = make_double2(z.x * scale, z.y * scale);
    }
    int32_t c[4];
    int64_t r = s;
    for (int d = 0; d < 4; ++d) {
        c[d] = (int32_t)(r % g.L[d]);
        r /= g.L[d];
    }
    store_record(base, prec, 1, 12, 0, (int32_t)cb_index(g, c[0], c[1], c[2], c[3]), v, 12);
}

// Zero a FERMION field (F16S scales set to 1), then put 1 at one component.
__global__ __launch_bounds__(256) void point_kernel(Geometry g, char* base, int32_t prec, int32_t target,
                                                    int32_t comp) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    double2 v[12];
    for (int k = 0; k < 12; ++k) v[k] = make_double2(s == target && k == comp ? 1.0 : 0.0, 0.0);
    store_record(base, prec, 1, 12, 0, (int32_t)s, v, 12);
}

}  // namespace

qdp_status fill_random_impl(Ctx* ctx, uint64_t f, int32_t kind, uint64_t seed, int32_t column, double scale) {
    Field* fd = find_field(ctx, f);
    if (!fd) return set_error(ctx, QDP_ERR_STATE, "fill_random: unknown field");
    const Geometry& g = find_lattice(ctx, fd->lattice)->geo;
    char* p;
    PinSet pins(ctx);
    if (kind == QDP_RANDOM_SU3) {
        if (fd->type != QDP_GAUGE) return set_error(ctx, QDP_ERR_TYPE, "fill_random SU3 needs a GAUGE field");
        QDP_CHECK(pins.add(f, false, &p));
        const int64_t n = 4 * g.V;
        hipLaunchKernelGGL(su3_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, g, p, fd->prec,
                           seed);
    } else if (kind == QDP_RANDOM_GAUSSIAN) {
        if (fd->type != QDP_FERMION) return set_error(ctx, QDP_ERR_TYPE, "fill_random GAUSSIAN needs a FERMION field");
        if (column < 0) return set_error(ctx, QDP_ERR_ARG, "fill_random: negative column");
        QDP_CHECK(pins.add(f, false, &p));
        hipLaunchKernelGGL(gaussian_kernel, dim3((unsigned)((g.V + 255) / 256)), dim3(256), 0, ctx->stream, g, p,
                           fd->prec, seed, column, scale);
    } else {
        return set_error(ctx, QDP_ERR_ARG, "fill_random: unknown kind %d", kind);
    }
    return check_launch(ctx, "fill_random kernel");
}

qdp_status fill_point_impl(Ctx* ctx, uint64_t f, int64_t site, int32_t spin, int32_t colour) {
    Field* fd = find_field(ctx, f);
    if (!fd) return set_error(ctx, QDP_ERR_STATE, "fill_point: unknown field");
    if (fd->type != QDP_FERMION) return set_error(ctx, QDP_ERR_TYPE, "fill_point needs a FERMION field");
    const Geometry& g = find_lattice(ctx, fd->lattice)->geo;
    if (site < 0 || site >= g.V || spin < 0 || spin > 3 || colour < 0 || colour > 2)
        return set_error(ctx, QDP_ERR_ARG, "fill_point: site/spin/colour out of range");
    int32_t c[4];
    int64_t r = site;
    for (int d = 0; d < 4; ++d) {
        c[d] = (int32_t)(r % g.L[d]);
        r /= g.L[d];
    }
    const int32_t cb = (int32_t)cb_index(g, c[0], c[1], c[2], c[3]);
    char* p;
    PinSet pins(ctx);
    QDP_CHECK(pins.add(f, false, &p));
    hipLaunchKernelGGL(point_kernel, dim3((unsigned)((g.V + 255) / 256)), dim3(256), 0, ctx->stream, g, p, fd->prec,
                       cb, 3 * spin + colour);
    return check_launch(ctx, "fill_point kernel");
}

}  // namespace qdpmi
