// Meson two-point contractions: the mesonic hadron spectrum (HAD, section 5
// and Figure 4 of the paper) for all 16 gamma bilinears,
//
//   C_n(t) = sum_{x: x_3 = t} Tr[ g5 S2(x)^dagger g5 Gamma_n S1(x) Gamma_n ].
//
// In the DeGrand-Rossi basis every Gamma_n is a signed permutation whose
// permutation sigma lies in the Klein four-group {id, (01)(23), (02)(13),
// (03)(12)}; the four Gammas sharing a sigma share the colour sums
//
//   G_sigma[a][b] = sum_{i,j colour} conj(S2[(a i),(b j)]) S1[(sigma a, i),(sigma b, j)]
//
// and C_n = sum_{a,b} P_n[a] Q_n[b] G_sigma[a][b] with P_n[a] = s_a Gamma_n[a, sigma a],
// Q_n[b] = s_b Gamma_n[sigma b, b], s = diag(g5).  One wavefront of a block
// handles one sigma for 64 sites; the four wavefronts read the same sites.
// Products and sums are FP64 (propagators grow like 2^N under smearing and
// |S|^2 leaves the FP32 range).  The time-slice sums are two-stage with a
// fixed order: bitwise repeatable.
#include <hip/hip_runtime.h>

#include <cstring>
#include <type_traits>
#include <vector>

#include "device.hpp"
#include "internal.hpp"

namespace qdpmi {

struct GammaDev {
    int8_t perm[4][4];     // sigma -> spin permutation
    int8_t members[4][4];  // sigma -> n values
    int8_t pcode[16][4];   // phase code of P_n[a]: i^code
    int8_t qcode[16][4];   // phase code of Q_n[b]
};

struct ContractArgs {
    Geometry g;
    const char* s1[12];
    const char* s2[12];
    double* partial;  // [Lt][nchunks][16][2]
    int32_t nchunks;
    int32_t pad;
};

// One 12-component column at one checkerboard site, as loaded: FP64 and FP32
// values, or F16S half2 values with the record scale (decoded when used, so
// an in-flight record takes 13 registers).  Products are formed in FP64.
template <int PREC>
struct RawCol {
    typename std::conditional<PREC == QDP_F64, double2, float2>::type v[12];
    __device__ __forceinline__ double2 at(int k) const { return make_double2(v[k].x, v[k].y); }
};
template <>
struct RawCol<QDP_F16S> {
    half2_t h[12];
    float scale;
    __device__ __forceinline__ double2 at(int k) const {
        const float2 f = f16s_decode(h[k], scale);
        return make_double2(f.x, f.y);
    }
};

template <int PREC, bool BUF>
__device__ __forceinline__ void load_column(const char* base, int32_t s, RawCol<PREC>& r) {
    if constexpr (PREC == QDP_F16S) {
        const FieldRef<half2_t, BUF> f(base);
        const FieldRef<float, BUF> sc(base);
        const int64_t so = site_off<half2_t>(s, tile_bytes(1, 12, QDP_F16S));
        r.scale = sc.load(12, so);
#pragma unroll
        for (int k = 0; k < 12; ++k) r.h[k] = f.load(k, so);
    } else {
        using T = typename std::remove_reference<decltype(r.v[0])>::type;
        const FieldRef<T, BUF> f(base);
        const int64_t so = site_off<T>(s, tile_bytes(1, 12, PREC));
#pragma unroll
        for (int k = 0; k < 12; ++k) r.v[k] = f.load(k, so);
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// i^code as (re, im), code mod 4.
__device__ __forceinline__ double2 unit_phase(int code) {
    code &= 3;
    return make_double2(code == 0 ? 1.0 : (code == 2 ? -1.0 : 0.0), code == 1 ? 1.0 : (code == 3 ? -1.0 : 0.0));
}

// Sites of one slice chunk for the Klein-group element SIGMA (spin
// permutation a -> a ^ SIGMA).  The source spin beta is the outer loop so
// only one column of G and the four correlators stay in registers.
template <int PREC, bool BUF, int SIGMA>
__device__ __forceinline__ void meson_sites(const ContractArgs& A, const GammaDev& gd, int t, int chunk, int lane,
                                            double2 C[4]) {
    const int64_t Vsh = A.g.Vsh;
    const int64_t Vs = 2 * Vsh;
    int n[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) n[m] = gd.members[SIGMA][m];
    for (int64_t l = (int64_t)chunk * 64 + lane; l < Vs; l += (int64_t)A.nchunks * 64) {
        const int64_t p = l >= Vsh ? 1 : 0;
        const int32_t s = (int32_t)(p * A.g.Vh + t * Vsh + (l - p * Vsh));
#pragma unroll
        for (int beta = 0; beta < 4; ++beta) {
            double2 G[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) G[x] = make_double2(0.0, 0.0);
            // the six columns of this source spin (three colours of S2 and
            // of S1) are requested before the arithmetic: one wait on memory
            // per source spin
            RawCol<PREC> c2[3], c1[3];
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                load_column<PREC, BUF>(A.s2[3 * beta + b], s, c2[b]);
                load_column<PREC, BUF>(A.s1[3 * (beta ^ SIGMA) + b], s, c1[b]);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
#pragma unroll
                for (int alpha = 0; alpha < 4; ++alpha)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        cmac_conj(G[alpha], c2[b].at(3 * alpha + c), c1[b].at(3 * (alpha ^ SIGMA) + c));
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
#pragma unroll
                for (int alpha = 0; alpha < 4; ++alpha) {
                    const double2 ph = unit_phase(gd.pcode[n[m]][alpha] + gd.qcode[n[m]][beta]);
                    cmac(C[m], ph, G[alpha]);
                }
            }
        }
    }
}

template <int PREC, bool BUF>
__global__ __launch_bounds__(256) void meson_kernel(ContractArgs a, GammaDev gd) {
    const int t = blockIdx.y;
    const int chunk = blockIdx.x;
    const int sigma = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    double2 C[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) C[m] = make_double2(0.0, 0.0);
    switch (sigma) {
        case 0: meson_sites<PREC, BUF, 0>(a, gd, t, chunk, lane, C); break;
        case 1: meson_sites<PREC, BUF, 1>(a, gd, t, chunk, lane, C); break;
        case 2: meson_sites<PREC, BUF, 2>(a, gd, t, chunk, lane, C); break;
        default: meson_sites<PREC, BUF, 3>(a, gd, t, chunk, lane, C); break;
    }
    __shared__ double red[4][4][2];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const double re = wave_sum(C[m].x);
        const double im = wave_sum(C[m].y);
        if (lane == 0) {
            red[sigma][m][0] = re;
            red[sigma][m][1] = im;
        }
    }
    __syncthreads();
    if (threadIdx.x < 16) {
        const int sg = threadIdx.x >> 2, m = threadIdx.x & 3;
        const int n = gd.members[sg][m];
        double* out = a.partial + (((int64_t)t * a.nchunks + chunk) * 16 + n) * 2;
        out[0] = red[sg][m][0];
        out[1] = red[sg][m][1];
    }
}

// out[(n * Lt + (t - t0 mod Lt)) * 2 + k] = sum over chunks, fixed order.
__global__ void meson_finish(const double* __restrict__ partial, int32_t Lt, int32_t nchunks,
                             uint32_t mask, int32_t t0, double* __restrict__ out) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 16 * Lt) return;
    const int n = idx / Lt, t = idx % Lt;
    double re = 0.0, im = 0.0;
    if (mask & (1u << n)) {
        for (int c = 0; c < nchunks; ++c) {
            const double* p = partial + (((int64_t)t * nchunks + c) * 16 + n) * 2;
            re += p[0];
            im += p[1];
        }
    }
    const int tr = ((t - t0) % Lt + Lt) % Lt;
    out[(n * Lt + tr) * 2] = re;
    out[(n * Lt + tr) * 2 + 1] = im;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

// DeGrand-Rossi gamma_1..gamma_4 as signed permutations: row r has its one
// nonzero entry i^code[r] in column perm[r].
namespace {
struct SignedPerm {
    int perm[4];
    int code[4];
};
const SignedPerm kGammaBasis[4] = {
    {{3, 2, 1, 0}, {1, 1, 3, 3}},  // gamma_1
    {{3, 2, 1, 0}, {2, 0, 0, 2}},  // gamma_2
    {{2, 3, 0, 1}, {1, 3, 3, 1}},  // gamma_3
    {{2, 3, 0, 1}, {0, 0, 0, 0}},  // gamma_4
};
SignedPerm sp_mul(const SignedPerm& A, const SignedPerm& B) {
    SignedPerm C;
    for (int r = 0; r < 4; ++r) {
        C.perm[r] = B.perm[A.perm[r]];
        C.code[r] = (A.code[r] + B.code[A.perm[r]]) & 3;
    }
    return C;
}
}  // namespace

void build_gamma_tables(Ctx* ctx) {
    const int klein[4][4] = {{0, 1, 2, 3}, {1, 0, 3, 2}, {2, 3, 0, 1}, {3, 2, 1, 0}};
    const int s_code[4] = {0, 0, 2, 2};  // diag(g5) = (1, 1, -1, -1)
    int count[4] = {0, 0, 0, 0};
    auto& T = ctx->gamma;
    std::memset(&T, 0, sizeof T);
    for (int sg = 0; sg < 4; ++sg)
        for (int i = 0; i < 4; ++i) T.group_perm[sg][i] = klein[sg][i];
    for (int n = 0; n < 16; ++n) {
        SignedPerm G{{0, 1, 2, 3}, {0, 0, 0, 0}};
        for (int k = 0; k < 4; ++k)
            if (n & (1 << k)) G = sp_mul(G, kGammaBasis[k]);
        int sg = 0;
        for (; sg < 4; ++sg)
            if (std::memcmp(G.perm, klein[sg], sizeof G.perm) == 0) break;
        T.group_members[sg][count[sg]++] = n;
        for (int a = 0; a < 4; ++a) {
            const int pc = (G.code[a] + s_code[a]) & 3;             // s_a Gamma[a, sigma a]
            const int qc = (G.code[G.perm[a]] + s_code[a]) & 3;     // s_b Gamma[sigma b, b]
            T.p_phase[n][a][0] = pc == 0 ? 1 : (pc == 2 ? -1 : 0);
            T.p_phase[n][a][1] = pc == 1 ? 1 : (pc == 3 ? -1 : 0);
            T.q_phase[n][a][0] = qc == 0 ? 1 : (qc == 2 ? -1 : 0);
            T.q_phase[n][a][1] = qc == 1 ? 1 : (qc == 3 ? -1 : 0);
        }
    }
}

namespace {
int phase_code(const double ph[2]) {
    if (ph[0] > 0.5) return 0;
    if (ph[1] > 0.5) return 1;
    if (ph[0] < -0.5) return 2;
    return 3;
}

template <bool BUF>
void* meson_func_buf(int prec) {
    switch (prec) {
        case QDP_F64: return reinterpret_cast<void*>(&meson_kernel<QDP_F64, BUF>);
        case QDP_F32: return reinterpret_cast<void*>(&meson_kernel<QDP_F32, BUF>);
        default: return reinterpret_cast<void*>(&meson_kernel<QDP_F16S, BUF>);
    }
}

void* meson_func(int prec, bool buf) { return buf ? meson_func_buf<true>(prec) : meson_func_buf<false>(prec); }
}  // namespace

qdp_status hadron_contract_impl(Ctx* ctx, const uint64_t* S1, const uint64_t* S2, uint32_t mask,
                                int32_t t0, int32_t j_decay, double* out) {
    if (j_decay != 3) return set_error(ctx, QDP_ERR_UNSUPPORTED, "contract: only j_decay = 3 (time)");
    uint64_t lat = 0;
    int32_t prec = -1;
    for (int side = 0; side < 2; ++side)
        for (int c = 0; c < 12; ++c) {
            Field* f = find_field(ctx, side ? S2[c] : S1[c]);
            if (!f) return set_error(ctx, QDP_ERR_STATE, "contract: unknown column handle");
            if (f->type != QDP_FERMION) return set_error(ctx, QDP_ERR_TYPE, "contract: columns must be FERMION");
            if (lat && f->lattice != lat) return set_error(ctx, QDP_ERR_LATTICE, "contract: columns on different lattices");
            if (prec >= 0 && f->prec != prec)
                return set_error(ctx, QDP_ERR_UNSUPPORTED, "contract: all 24 columns must share one precision");
            lat = f->lattice;
            prec = f->prec;
        }
    const Geometry g = find_lattice(ctx, lat)->geo;
    const int32_t Lt = g.L[3];
    const int64_t Vs = 2 * g.Vsh;
    int64_t nchunks = (8192 + Lt - 1) / Lt;
    nchunks = std::max<int64_t>(1, std::min<int64_t>(nchunks, (Vs + 63) / 64));

    PinSet pins(ctx);
    ContractArgs a{};
    a.g = g;
    for (int c = 0; c < 12; ++c) {
        char* p;
        QDP_CHECK(pins.add(S1[c], true, &p));
        a.s1[c] = p;
        QDP_CHECK(pins.add(S2[c], true, &p));
        a.s2[c] = p;
    }
    a.nchunks = (int32_t)nchunks;
    PoolTemp scratch;
    const size_t partial_bytes = sizeof(double) * 2 * 16 * (size_t)Lt * nchunks;
    const size_t out_bytes = sizeof(double) * 2 * 16 * (size_t)Lt;
    QDP_CHECK(scratch.alloc(ctx, (int64_t)(partial_bytes + out_bytes + 256)));
    a.partial = reinterpret_cast<double*>(scratch.ptr());
    double* d_out = reinterpret_cast<double*>(scratch.ptr() + ((partial_bytes + 255) & ~size_t(255)));

    GammaDev gd;
    for (int sg = 0; sg < 4; ++sg)
        for (int i = 0; i < 4; ++i) {
            gd.perm[sg][i] = (int8_t)ctx->gamma.group_perm[sg][i];
            gd.members[sg][i] = (int8_t)ctx->gamma.group_members[sg][i];
        }
    for (int n = 0; n < 16; ++n)
        for (int i = 0; i < 4; ++i) {
            gd.pcode[n][i] = (int8_t)phase_code(ctx->gamma.p_phase[n][i]);
            gd.qcode[n][i] = (int8_t)phase_code(ctx->gamma.q_phase[n][i]);
        }

    void* args[] = {&a, &gd};
    const bool buf = field_bytes(g, QDP_FERMION, prec) < (int64_t(1) << 32);
    QDP_HIP(ctx, hipLaunchKernel(meson_func(prec, buf), dim3((unsigned)nchunks, (unsigned)Lt), dim3(256), args, 0,
                                 ctx->stream));
    QDP_CHECK(check_launch(ctx, "meson kernel"));
    const int nthreads = 16 * Lt;
    hipLaunchKernelGGL(meson_finish, dim3((nthreads + 255) / 256), dim3(256), 0, ctx->stream, a.partial, Lt,
                       (int32_t)nchunks, mask, t0, d_out);
    QDP_CHECK(check_launch(ctx, "meson finish kernel"));
    double* host;
    QDP_CHECK(host_result_buffer(ctx, out_bytes, &host));
    QDP_HIP(ctx, hipMemcpyAsync(host, d_out, out_bytes, hipMemcpyDeviceToHost, ctx->stream));
    QDP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::memcpy(out, host, out_bytes);
    return QDP_OK;
}

}  // namespace qdpmi
