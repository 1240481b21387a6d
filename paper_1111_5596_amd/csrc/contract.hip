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
// Q_n[b] = s_b Gamma_n[sigma b, b], s = diag(g5).  F16S contractions run one
// wavefront per source colour (each column of a site read once per block;
// with momenta when S1 and S2 are the same columns); the other precisions
// and the momentum-projected contractions of two propagators run one
// wavefront per sigma, the four wavefronts of a block reading the same 64
// sites.  Momentum projection weights each site's traces by exp(-i p.x)
// before the slice sum; one launch carries up to four momenta.
// Products and sums are FP64 (propagators grow like 2^N under smearing and
// |S|^2 leaves the FP32 range).  The time-slice sums are two-stage with a
// fixed order: bitwise repeatable.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "device.hpp"
#include "internal.hpp"

namespace qdpmi {

// DeGrand-Rossi gamma_1..gamma_4 as signed permutations: row r has its one
// nonzero entry i^code[r] in column perm[r].  constexpr, so that the device
// code's index arithmetic on them folds at compile time.
struct SignedPerm {
    int perm[4];
    int code[4];
};
constexpr SignedPerm kGammaBasis[4] = {
    {{3, 2, 1, 0}, {1, 1, 3, 3}},  // gamma_1
    {{3, 2, 1, 0}, {2, 0, 0, 2}},  // gamma_2
    {{2, 3, 0, 1}, {1, 3, 3, 1}},  // gamma_3
    {{2, 3, 0, 1}, {0, 0, 0, 0}},  // gamma_4
};
constexpr SignedPerm sp_mul(const SignedPerm& A, const SignedPerm& B) {
    SignedPerm C{};
    for (int r = 0; r < 4; ++r) {
        C.perm[r] = B.perm[A.perm[r]];
        C.code[r] = (A.code[r] + B.code[A.perm[r]]) & 3;
    }
    return C;
}
constexpr SignedPerm kGamma5 =
    sp_mul(sp_mul(sp_mul(kGammaBasis[0], kGammaBasis[1]), kGammaBasis[2]), kGammaBasis[3]);
// charge conjugation C = gamma_2 gamma_4 times gamma_5
constexpr SignedPerm kCg5 = sp_mul(sp_mul(kGammaBasis[1], kGammaBasis[3]), kGamma5);
// Hermitian conjugate and transpose of a signed permutation
constexpr SignedPerm sp_adj(const SignedPerm& A) {
    SignedPerm C{};
    for (int r = 0; r < 4; ++r) {
        C.perm[A.perm[r]] = r;
        C.code[A.perm[r]] = (4 - A.code[r]) & 3;
    }
    return C;
}
constexpr SignedPerm sp_trans(const SignedPerm& A) {
    SignedPerm C{};
    for (int r = 0; r < 4; ++r) {
        C.perm[A.perm[r]] = r;
        C.code[A.perm[r]] = A.code[r];
    }
    return C;
}
constexpr SignedPerm sp_neg(const SignedPerm& A) {
    SignedPerm C = A;
    for (int r = 0; r < 4; ++r) C.code[r] = (A.code[r] + 2) & 3;
    return C;
}
// diquark matrices at the sink (G) and the source (G' = gamma_4 G^dagger gamma_4^T):
// proton C gamma_5 (G' = -C gamma_5), Delta++ C gamma_mu for mu = 1, 2, 3
constexpr SignedPerm kCgamma[3] = {sp_mul(sp_mul(kGammaBasis[1], kGammaBasis[3]), kGammaBasis[0]),
                                   sp_mul(sp_mul(kGammaBasis[1], kGammaBasis[3]), kGammaBasis[1]),
                                   sp_mul(sp_mul(kGammaBasis[1], kGammaBasis[3]), kGammaBasis[2])};
constexpr SignedPerm source_diquark(const SignedPerm& G) {
    return sp_mul(sp_mul(kGammaBasis[3], sp_adj(G)), sp_trans(kGammaBasis[3]));
}
constexpr SignedPerm kGamma4 = kGammaBasis[3];

// Gamma_n = gamma_1^b0 gamma_2^b1 gamma_3^b2 gamma_4^b3 (b_k the bits of n)
constexpr SignedPerm gamma_n(int n) {
    SignedPerm G{{0, 1, 2, 3}, {0, 0, 0, 0}};
    for (int k = 0; k < 4; ++k)
        if (n & (1 << k)) G = sp_mul(G, kGammaBasis[k]);
    return G;
}

// The meson contraction's tables, derived at compile time from the signed
// permutations above: Gamma_n maps spin a to a ^ sigma (sigma = its row 0's
// column); members[sigma] lists the four n sharing sigma; P_n[a] =
// s_a Gamma_n[a, a ^ sigma] = i^pcode, Q_n[b] = s_b Gamma_n[b ^ sigma, b] =
// i^qcode, s = diag(gamma_5) = (1, 1, -1, -1).
struct MesonTables {
    int members[4][4];
    int pcode[16][4];
    int qcode[16][4];
};
constexpr MesonTables make_meson_tables() {
    MesonTables T{};
    int count[4] = {0, 0, 0, 0};
    const int s_code[4] = {0, 0, 2, 2};
    for (int n = 0; n < 16; ++n) {
        const SignedPerm G = gamma_n(n);
        const int sg = G.perm[0];
        T.members[sg][count[sg]++] = n;
        for (int a = 0; a < 4; ++a) {
            T.pcode[n][a] = (G.code[a] + s_code[a]) & 3;
            T.qcode[n][a] = (G.code[G.perm[a]] + s_code[a]) & 3;
        }
    }
    return T;
}
__device__ constexpr MesonTables kMesonTables = make_meson_tables();
// every Gamma_n permutes spins by an element of the Klein group a -> a ^ sigma
constexpr bool klein_grouping() {
    for (int n = 0; n < 16; ++n) {
        const SignedPerm G = gamma_n(n);
        for (int a = 0; a < 4; ++a)
            if (G.perm[a] != (a ^ G.perm[0])) return false;
    }
    return true;
}
static_assert(klein_grouping(), "DeGrand-Rossi Gamma_n are signed Klein-group permutations");

struct ContractArgs {
    Geometry g;
    const char* s1[12];
    const char* s2[12];
    double* partial;  // [Lt][nchunks][momenta of the launch][16][2]
    int32_t nchunks;
    int32_t pad;
    int32_t mom[4][3];  // integer momenta k of the launch, p_i = 2 pi k_i / L_i
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
    // the stored half values without the record scale
    __device__ __forceinline__ double2 stored(int k) const {
        return make_double2((double)(float)h[k].x, (double)(float)h[k].y);
    }
};

// re(conj(x) y) + c = x.x y.x + x.y y.y + c and im(conj(x) y) + c =
// -x.y y.x + x.x y.y + c for half2 x, y: products exact, one FP32 rounding
// per step (v_dot2_f32_f16; the imaginary part takes (-x.y, x.x), an exact
// swap and sign change of x).
__device__ __forceinline__ float dot2_conj_re(half2_t x, half2_t y, float c) {
    return __builtin_amdgcn_fdot2(x, y, c, false);
}
__device__ __forceinline__ float dot2_conj_im(half2_t x, half2_t y, float c) {
    return __builtin_amdgcn_fdot2(half2_t{(_Float16)(-x.y), x.x}, y, c, false);
}

// One column at one site: 16-byte chunk loads (3 for F16S, 6 for F32, 12 for
// F64) and, for F16S, the record scale.
template <int PREC, bool BUF>
__device__ __forceinline__ void load_column(const char* base, int32_t s, RawCol<PREC>& r) {
    const int64_t tb = tile_bytes(1, 12, PREC);
    const ChunkRef<BUF> f(base);
    const int64_t so16 = tile_site_offset(tb, 16, s);
    if constexpr (PREC == QDP_F16S) {
        r.scale = FieldRef<float, BUF>(base).load(12, site_off<float>(s, tb));
        load_elems<0, 12>(f, so16, r.h);
    } else {
        load_elems<0, 12>(f, so16, r.v);
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// z * i^k (k mod 4): for k known at compile time a swap and signs.
__device__ __forceinline__ double2 times_ik(double2 z, int k) {
    switch (k & 3) {
        case 0: return z;
        case 1: return make_double2(-z.y, z.x);
        case 2: return make_double2(-z.x, -z.y);
        default: return make_double2(z.y, -z.x);
    }
}

// Spatial coordinates of index l within the sites of time slice t (l = p Vsh
// + x/2 + (Lx/2)(y + Ly z) for the site of parity p; the parity fixes the low
// bit of x).  32-bit arithmetic: a time slice holds fewer than 2^31 sites.
__device__ __forceinline__ void slice_coords(const Geometry& g, uint32_t l, int32_t t, int32_t c[3]) {
    const uint32_t Vsh = (uint32_t)g.Vsh, Lxh = (uint32_t)g.Lxh, Ly = (uint32_t)g.L[1];
    const uint32_t p = l >= Vsh ? 1u : 0u;
    const uint32_t i = l - p * Vsh;
    const uint32_t yz = i / Lxh, z = yz / Ly;
    const uint32_t y = yz - z * Ly, xh = i - yz * Lxh;
    c[0] = (int32_t)(2 * xh + ((p + y + z + (uint32_t)t) & 1u));
    c[1] = (int32_t)y;
    c[2] = (int32_t)z;
}

// exp(-i p.x) for integer momentum k at spatial coordinates c: the phase
// angle is reduced exactly to a fraction num / (Lx Ly Lz) of a turn first
// (each k_i c_i mod L_i, k_i reduced mod L_i first, so every product and
// partial sum fits 32 bits: L_i^2 < 2^31 and the sum stays below 2 Lx Ly Lz).
__device__ __forceinline__ double2 plane_wave(const Geometry& g, const int32_t k[3], const int32_t c[3]) {
    const uint32_t M = (uint32_t)g.L[0] * (uint32_t)g.L[1] * (uint32_t)g.L[2];
    uint32_t num = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int32_t L = g.L[i];
        const uint32_t kr = (uint32_t)(((k[i] % L) + L) % L);
        const uint32_t r = (kr * (uint32_t)c[i]) % (uint32_t)L;
        num += r * (M / (uint32_t)L);
        if (num >= M) num -= M;
    }
    double sn, cs;
    sincospi(-2.0 * ((double)num / (double)M), &sn, &cs);
    return make_double2(cs, sn);
}

// Sites of one slice chunk for the Klein-group element SIGMA (spin
// permutation a -> a ^ SIGMA).  The source spin beta is the outer loop so
// only one column of G and the four correlators stay in registers.  NMOM = 0:
// zero momentum, C[m] accumulates the traces directly; NMOM > 0: a site's
// traces are complete first, then C[4 q + m] += exp(-i p_q.x) trace_m.
template <int PREC, bool BUF, int SIGMA, int NMOM>
__device__ __forceinline__ void meson_sites(const ContractArgs& A, int t, int chunk, int lane, double2* C) {
    const int64_t Vsh = A.g.Vsh;
    const int64_t Vs = 2 * Vsh;
    for (int64_t l = (int64_t)chunk * 64 + lane; l < Vs; l += (int64_t)A.nchunks * 64) {
        const int64_t p = l >= Vsh ? 1 : 0;
        const int32_t s = (int32_t)(p * A.g.Vh + t * Vsh + (l - p * Vsh));
        double2 site_tr[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) site_tr[m] = make_double2(0.0, 0.0);
        double2* acc = NMOM > 0 ? site_tr : C;
        // beta_c: a std::integral_constant (phases folded at compile time)
        // or, with momenta, a plain int (a rolled loop keeps the registers
        // of one source spin live at a time)
        auto source_spin = [&](auto beta_c) {
            const int beta = beta_c;
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
                if constexpr (PREC == QDP_F16S) {
                    // colour sums of the stored half values, conj(a) b summed
                    // over the three colours by v_dot2 (every product of two
                    // halves is exact in FP32, each sum rounds once to
                    // FP32: 2^-24 of the partial sum, which is at most 3 in
                    // magnitude, so no range is lost); then both record
                    // scales at once in FP64 (powers of two, the range of
                    // the smeared propagator) and every sum after in FP64
                    const double sc = (double)c2[b].scale * (double)c1[b].scale;
#pragma unroll
                    for (int alpha = 0; alpha < 4; ++alpha) {
                        float re = 0.f, im = 0.f;
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            const half2_t x = c2[b].h[3 * alpha + c], y = c1[b].h[3 * (alpha ^ SIGMA) + c];
                            re = dot2_conj_re(x, y, re);
                            im = dot2_conj_im(x, y, im);
                        }
                        G[alpha].x = fmadd(sc, (double)re, G[alpha].x);
                        G[alpha].y = fmadd(sc, (double)im, G[alpha].y);
                    }
                } else {
#pragma unroll
                    for (int alpha = 0; alpha < 4; ++alpha)
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            cmac_conj(G[alpha], c2[b].at(3 * alpha + c), c1[b].at(3 * (alpha ^ SIGMA) + c));
                }
            }
            // C_n += P_n[alpha] Q_n[beta] G[alpha]: a phase i^k known at
            // compile time, so a swap and signs folded into the additions
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int n = kMesonTables.members[SIGMA][m];
#pragma unroll
                for (int alpha = 0; alpha < 4; ++alpha) {
                    const double2 z =
                        times_ik(G[alpha], kMesonTables.pcode[n][alpha] + kMesonTables.qcode[n][beta]);
                    acc[m].x += z.x;
                    acc[m].y += z.y;
                }
            }
        };
        if constexpr (NMOM > 0) {
            // kept rolled: unrolled, the compiler hoists several source
            // spins' loads and spills them when the momentum tail follows
#pragma unroll 1
            for (int beta = 0; beta < 4; ++beta) source_spin(beta);
        } else {
            source_spin(std::integral_constant<int, 0>{});
            source_spin(std::integral_constant<int, 1>{});
            source_spin(std::integral_constant<int, 2>{});
            source_spin(std::integral_constant<int, 3>{});
        }
        if constexpr (NMOM > 0) {
            int32_t c[3];
            slice_coords(A.g, (uint32_t)l, t, c);
#pragma unroll
            for (int q = 0; q < NMOM; ++q) {
                const double2 w = plane_wave(A.g, A.mom[q], c);
#pragma unroll
                for (int m = 0; m < 4; ++m) cmac(C[4 * q + m], w, site_tr[m]);
            }
        }
    }
}

template <int PREC, bool BUF, int NMOM>
__global__ __launch_bounds__(256) void meson_kernel(ContractArgs a) {
    constexpr int NQ = NMOM > 0 ? NMOM : 1;
    const int t = blockIdx.y;
    const int chunk = blockIdx.x;
    const int sigma = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    double2 C[4 * NQ];
#pragma unroll
    for (int m = 0; m < 4 * NQ; ++m) C[m] = make_double2(0.0, 0.0);
    switch (sigma) {
        case 0: meson_sites<PREC, BUF, 0, NMOM>(a, t, chunk, lane, C); break;
        case 1: meson_sites<PREC, BUF, 1, NMOM>(a, t, chunk, lane, C); break;
        case 2: meson_sites<PREC, BUF, 2, NMOM>(a, t, chunk, lane, C); break;
        default: meson_sites<PREC, BUF, 3, NMOM>(a, t, chunk, lane, C); break;
    }
    __shared__ double red[4][4 * NQ][2];
#pragma unroll
    for (int m = 0; m < 4 * NQ; ++m) {
        const double re = wave_sum(C[m].x);
        const double im = wave_sum(C[m].y);
        if (lane == 0) {
            red[sigma][m][0] = re;
            red[sigma][m][1] = im;
        }
    }
    __syncthreads();
    if (threadIdx.x < 16 * NQ) {
        const int q = threadIdx.x >> 4, sg = (threadIdx.x >> 2) & 3, m = threadIdx.x & 3;
        const int n = kMesonTables.members[sg][m];
        double* out = a.partial + ((((int64_t)t * a.nchunks + chunk) * NQ + q) * 16 + n) * 2;
        out[0] = red[sg][4 * q + m][0];
        out[1] = red[sg][4 * q + m][1];
    }
}

// ---------------------------------------------------------------------------
// Zero-momentum F16S contraction, one wavefront per source colour
// ---------------------------------------------------------------------------
// Within a Klein coset the four bilinears differ only by signs that depend on
// a ^ b: P_n[a] Q_n[b] = B_sigma[a][b] f_n(a ^ b), B_sigma the phases of the
// coset's first member and f_n(k) = +1 or -1 (checked at compile time).  So
// the slice sum needs only H_sigma[k] = sum_{a ^ b = k} B_sigma[a][b]
// G_sigma[a][b], 16 complex numbers, and C_n = sum_k f_n(k) H_sigma(n)[k]
// once per block.  Every colour sum of G lands in one H with a phase i^m
// known at compile time: no per-bilinear folding per site.
//
// The source colour j of G's sum splits the work: wavefront j of a block
// loads, for its 64 sites, the four S2 columns (beta, j) and the four S1
// columns (beta', j) -- four when S1 and S2 are the same columns -- and forms
// all 16 pairs (beta, beta'), sigma = beta ^ beta'.  Every column of a site
// is read once per block, where the one-wavefront-per-sigma kernel reads it
// four times (or eight, aliased).
struct MesonFold {
    int base[4][4][4];  // [sigma][a][b]: phase code of P_n0[a] Q_n0[b], n0 = members[sigma][0]
    int sign[16][4];    // [n][k]: f_n(k)
    int sigma_of[16];   // [n]: the coset of Gamma_n
};
constexpr MesonFold make_meson_fold() {
    MesonFold F{};
    const MesonTables T = make_meson_tables();
    for (int sg = 0; sg < 4; ++sg) {
        const int n0 = T.members[sg][0];
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) F.base[sg][a][b] = (T.pcode[n0][a] + T.qcode[n0][b]) & 3;
        for (int m = 0; m < 4; ++m) {
            const int n = T.members[sg][m];
            F.sigma_of[n] = sg;
            for (int k = 0; k < 4; ++k) F.sign[n][k] = ((T.pcode[n][0] + T.qcode[n][k] - F.base[sg][0][k]) & 3) ? -1 : 1;
        }
    }
    return F;
}
__device__ constexpr MesonFold kMesonFold = make_meson_fold();
constexpr bool meson_fold_exact() {
    const MesonTables T = make_meson_tables();
    const MesonFold F = make_meson_fold();
    for (int sg = 0; sg < 4; ++sg)
        for (int m = 0; m < 4; ++m) {
            const int n = T.members[sg][m];
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) {
                    const int d = (T.pcode[n][a] + T.qcode[n][b] - F.base[sg][a][b]) & 3;
                    if (d != (F.sign[n][a ^ b] == 1 ? 0 : 2)) return false;
                }
        }
    return true;
}
static_assert(meson_fold_exact(), "bilinears of a Klein coset differ by signs f_n(a ^ b)");

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// h += i^M sc (re + i im) with the phase folded into the signs
template <int M>
__device__ __forceinline__ void add_phased(double2& h, double sc, float re, float im) {
    const double r = (double)re, i = (double)im;
    if constexpr (M == 0) {
        h.x = fmadd(sc, r, h.x);
        h.y = fmadd(sc, i, h.y);
    } else if constexpr (M == 1) {
        h.x = fmadd(-sc, i, h.x);
        h.y = fmadd(sc, r, h.y);
    } else if constexpr (M == 2) {
        h.x = fmadd(-sc, r, h.x);
        h.y = fmadd(-sc, i, h.y);
    } else {
        h.x = fmadd(sc, i, h.x);
        h.y = fmadd(-sc, r, h.y);
    }
}

// The pair (S2 column (BETA, j), S1 column (BETA2, j)) of one site: for each
// sink spin a, the colour sum of conj(S2[(a i),(BETA j)]) S1[(a ^ sigma, i),
// (BETA2 j)] from the stored halves by v_dot2 (products exact, FP32 sums as
// in the one-wavefront-per-sigma kernel), then both record scales in FP64.
template <int BETA, int BETA2>
__device__ __forceinline__ void meson_pair_f16s(const RawCol<QDP_F16S>& x, const RawCol<QDP_F16S>& y,
                                                double2 (&H)[4][4]) {
    constexpr int SIGMA = BETA ^ BETA2;
    const double sc = (double)x.scale * (double)y.scale;
    static_for<0, 4>([&](auto a_c) {
        constexpr int a = decltype(a_c)::value;
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const half2_t xh = x.h[3 * a + c], yh = y.h[3 * (a ^ SIGMA) + c];
            re = dot2_conj_re(xh, yh, re);
            im = dot2_conj_im(xh, yh, im);
        }
        add_phased<kMesonFold.base[SIGMA][a][BETA]>(H[SIGMA][a ^ BETA], sc, re, im);
    });
}

// H += the 16 pairs of source colour j at site s
template <bool BUF, bool ALIAS>
__device__ __forceinline__ void colour_site_sums(const ContractArgs& A, int32_t s, int j, double2 (&H)[4][4]) {
    RawCol<QDP_F16S> x[4], y[ALIAS ? 1 : 4];
#pragma unroll
    for (int beta = 0; beta < 4; ++beta) {
        load_column<QDP_F16S, BUF>(A.s2[3 * beta + j], s, x[beta]);
        if constexpr (!ALIAS) load_column<QDP_F16S, BUF>(A.s1[3 * beta + j], s, y[beta]);
    }
    static_for<0, 4>([&](auto b_c) {
        constexpr int BETA = decltype(b_c)::value;
        static_for<0, 4>([&](auto b2_c) {
            constexpr int BETA2 = decltype(b2_c)::value;
            if constexpr (ALIAS)
                meson_pair_f16s<BETA, BETA2>(x[BETA], x[BETA2], H);
            else
                meson_pair_f16s<BETA, BETA2>(x[BETA], y[BETA2], H);
        });
        // keep one S2 column's operands live at a time
        __builtin_amdgcn_sched_barrier(0);
    });
}

template <bool BUF, bool ALIAS>
__global__ __launch_bounds__(192) __attribute__((amdgpu_waves_per_eu(2))) void meson_colour_kernel(ContractArgs A) {
    const int t = blockIdx.y;
    const int chunk = blockIdx.x;
    const int j = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // source colour of this wavefront
    const int lane = threadIdx.x & 63;
    double2 H[4][4];
#pragma unroll
    for (int sg = 0; sg < 4; ++sg)
#pragma unroll
        for (int k = 0; k < 4; ++k) H[sg][k] = make_double2(0.0, 0.0);
    const int64_t Vsh = A.g.Vsh;
    const int64_t Vs = 2 * Vsh;
    for (int64_t l = (int64_t)chunk * 64 + lane; l < Vs; l += (int64_t)A.nchunks * 64) {
        const int64_t p = l >= Vsh ? 1 : 0;
        const int32_t s = (int32_t)(p * A.g.Vh + t * Vsh + (l - p * Vsh));
        colour_site_sums<BUF, ALIAS>(A, s, j, H);
    }
    // block sum over the three colours (fixed order), then the bilinears
    __shared__ double red[3][16][2];
#pragma unroll
    for (int sg = 0; sg < 4; ++sg)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double re = wave_sum(H[sg][k].x);
            const double im = wave_sum(H[sg][k].y);
            if (lane == 0) {
                red[j][4 * sg + k][0] = re;
                red[j][4 * sg + k][1] = im;
            }
        }
    __syncthreads();
    if (threadIdx.x < 32) {
        const int n = threadIdx.x >> 1, ri = threadIdx.x & 1;
        const int sg = kMesonFold.sigma_of[n];
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double hk = (red[0][4 * sg + k][ri] + red[1][4 * sg + k][ri]) + red[2][4 * sg + k][ri];
            v += kMesonFold.sign[n][k] * hk;
        }
        A.partial[(((int64_t)t * A.nchunks + chunk) * 16 + n) * 2 + ri] = v;
    }
}

// Momentum-projected F16S contraction, four momenta per launch.  Waves 0..2
// form a site's 16 sums H_sigma[k] for their source colour as above while
// wave 3 forms the site's four plane waves; the three colours' sums and the
// phases meet in LDS, and wavefront q (0..3) adds the sums (fixed order) and
// weights them by the plane wave of momentum q at the site, so each site's
// phase is computed once per momentum.  C_n = sum_k f_n(k)
// H_sigma(n)[k] once per block, as at zero momentum.
constexpr int kColourMomenta = 4;
template <bool BUF, bool ALIAS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void meson_colour_mom_kernel(ContractArgs A) {
    const int t = blockIdx.y;
    const int chunk = blockIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // colour (w < 3) and momentum
    const int lane = threadIdx.x & 63;
    __shared__ double2 hs[3][16][64];
    __shared__ double2 phs[kColourMomenta][64];
    double2 C[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) C[e] = make_double2(0.0, 0.0);
    const int64_t Vsh = A.g.Vsh;
    const int64_t Vs = 2 * Vsh;
    // every wavefront walks the same sites: the trip count is uniform over
    // the block (barriers inside); lanes past the slice take zeros
    for (int64_t base = (int64_t)chunk * 64; base < Vs; base += (int64_t)A.nchunks * 64) {
        const int64_t l = base + lane;
        const bool active = l < Vs;
        const int64_t lc = active ? l : Vs - 1;
        const int64_t p = lc >= Vsh ? 1 : 0;
        const int32_t s = (int32_t)(p * A.g.Vh + t * Vsh + (lc - p * Vsh));
        if (w < 3) {
            double2 H[4][4];
#pragma unroll
            for (int sg = 0; sg < 4; ++sg)
#pragma unroll
                for (int k = 0; k < 4; ++k) H[sg][k] = make_double2(0.0, 0.0);
            colour_site_sums<BUF, ALIAS>(A, s, w, H);
#pragma unroll
            for (int e = 0; e < 16; ++e) hs[w][e][lane] = active ? H[e >> 2][e & 3] : make_double2(0.0, 0.0);
        } else {
            // meanwhile the fourth wavefront forms the sites' four plane waves
            int32_t c[3];
            slice_coords(A.g, (uint32_t)lc, t, c);
#pragma unroll
            for (int q = 0; q < kColourMomenta; ++q) phs[q][lane] = plane_wave(A.g, A.mom[q], c);
        }
        __syncthreads();
        const double2 ph = phs[w][lane];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const double2 a = hs[0][e][lane], b = hs[1][e][lane], d = hs[2][e][lane];
            const double2 h = make_double2((a.x + b.x) + d.x, (a.y + b.y) + d.y);
            cmac(C[e], ph, h);
        }
        __syncthreads();
    }
    __shared__ double red[kColourMomenta][16][2];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const double re = wave_sum(C[e].x);
        const double im = wave_sum(C[e].y);
        if (lane == 0) {
            red[w][e][0] = re;
            red[w][e][1] = im;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * 16 * kColourMomenta) {
        const int q = threadIdx.x >> 5, n = (threadIdx.x >> 1) & 15, ri = threadIdx.x & 1;
        const int sg = kMesonFold.sigma_of[n];
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) v += kMesonFold.sign[n][k] * red[q][4 * sg + k][ri];
        A.partial[((((int64_t)t * A.nchunks + chunk) * kColourMomenta + q) * 16 + n) * 2 + ri] = v;
    }
}

// out[((q * 16 + n) * Lt + (t - t0 mod Lt)) * 2 + k] = sum over chunks, fixed
// order, for the nq momenta of a launch (nq = 1 at zero momentum).
__global__ void meson_finish(const double* __restrict__ partial, int32_t Lt, int32_t nchunks, int32_t nq,
                             uint32_t mask, int32_t t0, double* __restrict__ out) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nq * 16 * Lt) return;
    const int q = idx / (16 * Lt), n = (idx / Lt) % 16, t = idx % Lt;
    double re = 0.0, im = 0.0;
    if (mask & (1u << n)) {
        for (int c = 0; c < nchunks; ++c) {
            const double* p = partial + ((((int64_t)t * nchunks + c) * nq + q) * 16 + n) * 2;
            re += p[0];
            im += p[1];
        }
    }
    const int tr = ((t - t0) % Lt + Lt) % Lt;
    out[((q * 16 + n) * Lt + tr) * 2] = re;
    out[((q * 16 + n) * Lt + tr) * 2 + 1] = im;
}

// ---------------------------------------------------------------------------
// Proton two-point function (the baryon part of HAD):
//   C(t) = sum_{x: x_3 = t} sum_{g g'} P_{g'g} <chi_g(x) chibar_g'(0)>,
//   chi = eps_abc (u_a^T Cg5 d_b) u_c, chibar its Dirac adjoint (so the source
//   diquark matrix is G' = -Cg5), P = (1 + parity gamma_4) / 2.
// With spin blocks X^{aa'}_{rr'} = S[(r a),(r' a')] and M^{bb'} = Cg5 D^{bb'} G',
// Wick's direct and exchange terms summed against eps eps' collapse, for the
// two colours {x < y} other than b and {x' < y'} other than b', to
//   C = sum_{b b'} s_b s_b' [ f(U^{xx'}, U^{yy'}) - f(U^{xy'}, U^{yx'}) ],
//   f(X, Y) = Tr[P Y] <X, M> + Tr[P X] <Y, M> + <X P Y, M> + <Y P X, M>,
// where <A, B> = sum_{rr'} A_{rr'} B_{rr'} and s_b is the sign of the colour
// permutation (x, b, y).  One thread per site, nine (b, b') steps each
// reading five spin blocks; values decoded to FP64, products and sums FP64.
// ---------------------------------------------------------------------------

struct BaryonArgs {
    Geometry g;
    const char* su[12];
    const char* sd[12];
    double* partial;  // [Lt][nchunks][2]
    int32_t nchunks;
    int32_t parity;
};


// X[r][r'] = component (r, A) of column 3 r' + AP at checkerboard site s.
// Component 3 r + A lies in chunk (3 r + A) / CE at position (3 r + A) % CE
// (CE = components per 16-byte chunk), known at compile time: the chunks a
// column contributes are loaded whole (the compiler merges repeated loads
// of one chunk) and the components picked out of them.
template <int PREC, bool BUF, int A, int AP>
__device__ __forceinline__ void load_block(const char* const* cols, int32_t s, double2 X[4][4]) {
    using T = typename std::conditional<PREC == QDP_F64, double2,
                                        typename std::conditional<PREC == QDP_F32, float2, half2_t>::type>::type;
    constexpr int CE = 16 / sizeof(T);
    const int64_t tb = tile_bytes(1, 12, PREC);
    const int64_t so16 = tile_site_offset(tb, 16, s);
#pragma unroll
    for (int rp = 0; rp < 4; ++rp) {
        const char* base = cols[3 * rp + AP];
        const ChunkRef<BUF> f(base);
        float scale = 1.f;
        if constexpr (PREC == QDP_F16S) scale = FieldRef<float, BUF>(base).load(12, site_off<float>(s, tb));
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = 3 * r + A;
            const Chunk<T> c = __builtin_bit_cast(Chunk<T>, f.load(e / CE, so16));
            const T v = c.v[e % CE];
            if constexpr (PREC == QDP_F16S) {
                // an FMA with a +0 addend converts and scales in one mixed-precision
                // instruction (exact: the scale is a power of two)
                X[r][rp] = make_double2(__builtin_fmaf((float)v.x, scale, 0.0f), __builtin_fmaf((float)v.y, scale, 0.0f));
            } else {
                X[r][rp] = make_double2(v.x, v.y);
            }
        }
    }
}

// F16S propagator of 64 sites staged in LDS: one 256-byte row (64 lanes x
// one half2) per component e of column j (row 12 j + e), then one row of FP32
// record scales per column (row 144 + j).  The rows are filled by the
// buffer-to-LDS copy path (4 bytes per lane, no registers), so that the nine
// colour steps read the blocks they use from LDS: a site's 12 columns are
// fetched once instead of once per block that uses them (each u block enters
// four colour steps).
constexpr int kBaryonLdsRows = 12 * 12 + 12;
constexpr int kBaryonLdsPairBytes = kBaryonLdsRows * 256;

typedef __attribute__((address_space(3))) void baryon_lds_void_t;

// Copies columns 6 half .. 6 half + 5 at site s (this lane's) into the rows
// at `rows` (the two wavefronts sharing the rows copy one half each); the
// copies are complete after the wait below.
__device__ __forceinline__ void stage_propagator_half_f16s(const char* const* cols, int32_t s, char* rows, int half) {
    const int64_t tb = tile_bytes(1, 12, QDP_F16S);
    const int32_t vo16 = (int32_t)tile_site_offset(tb, 16, s), vo4 = (int32_t)site_off<float>(s, tb);
#pragma unroll
    for (int jj = 0; jj < 6; ++jj) {
        const int j = 6 * half + jj;
        const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(cols[j]);
#pragma unroll
        for (int e = 0; e < 12; ++e)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (baryon_lds_void_t*)(rows + (12 * j + e) * 256), 4, vo16,
                                                     (e / 4) * 1024 + (e % 4) * 4, 0, 0);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (baryon_lds_void_t*)(rows + (144 + j) * 256), 4, vo4, 12 * 256,
                                                 0, 0);
    }
}

// Waits until this wavefront's copies into LDS have landed; the memory
// clobber keeps the compiler from moving LDS reads above the wait.
__device__ __forceinline__ void wait_staged() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// load_block from the staged rows (`lane_rows` = the rows' base + 4 lane).
template <int A, int AP>
__device__ __forceinline__ void load_block_lds(const char* lane_rows, double2 X[4][4]) {
#pragma unroll
    for (int rp = 0; rp < 4; ++rp) {
        const int j = 3 * rp + AP;
        const float scale = *reinterpret_cast<const float*>(lane_rows + (144 + j) * 256);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const half2_t v = *reinterpret_cast<const half2_t*>(lane_rows + (12 * j + 3 * r + A) * 256);
            X[r][rp] = make_double2(__builtin_fmaf((float)v.x, scale, 0.0f), __builtin_fmaf((float)v.y, scale, 0.0f));
        }
    }
}

// A block of u (D = false) or d (D = true): from the staged rows when LDS
// holds that propagator (SRC = 1: u; SRC = 2: u, which is also d), else
// from memory.
template <int PREC, bool BUF, int SRC, bool D, int A, int AP>
__device__ __forceinline__ void get_block(const BaryonArgs& a, int32_t s, const char* lane_rows, double2 X[4][4]) {
    if constexpr (SRC == 2 || (SRC == 1 && !D))
        load_block_lds<A, AP>(lane_rows, X);
    else
        load_block<PREC, BUF, A, AP>(D ? a.sd : a.su, s, X);
}

__device__ __forceinline__ double2 cmul(double2 u, double2 v) {
    double2 z = make_double2(0.0, 0.0);
    cmac(z, u, v);
    return z;
}

// Tr[P Y] with P = 1/2 + hp gamma_4 (hp = parity / 2).
__device__ __forceinline__ double2 trace_p(const double2 Y[4][4], double hp) {
    double2 d = make_double2(0.0, 0.0), o = make_double2(0.0, 0.0);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        d.x += Y[g][g].x;
        d.y += Y[g][g].y;
        const double2 z = times_ik(Y[kGamma4.perm[g]][g], kGamma4.code[g]);
        o.x += z.x;
        o.y += z.y;
    }
    return make_double2(0.5 * d.x + hp * o.x, 0.5 * d.y + hp * o.y);
}

__device__ __forceinline__ double2 inner_plain(const double2 A[4][4], const double2 B[4][4]) {
    double2 z = make_double2(0.0, 0.0);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) cmac(z, A[r][c], B[r][c]);
    return z;
}

// <X P Y, M> = sum_{r, g} (X P)_{rg} (Y M^T)_{gr}.
// Tr(X P Y M^T) with the rank-2 projector P = (1 + 2 hp gamma_4) / 2 =
// (1/2) sum_k u_k u_k^T, u_k = e_k + s e_{k+2} (s = 2 hp = +1 or -1; gamma_4
// swaps spins 0 <-> 2 and 1 <-> 3 with unit entries): (1/2) sum_k
// (Y^T u_k) . M^T (X u_k), 2 x 20 complex MACs instead of 80.
constexpr bool gamma4_swaps_pairs() {
    for (int g = 0; g < 4; ++g)
        if (kGamma4.perm[g] != (g ^ 2) || kGamma4.code[g] != 0) return false;
    return true;
}
static_assert(gamma4_swaps_pairs(), "DeGrand-Rossi gamma_4 pairs spins 0, 2 and 1, 3 with unit entries");
__device__ __forceinline__ double2 xpy_m(const double2 X[4][4], const double2 Y[4][4], const double2 M[4][4],
                                        double hp) {
    const double sg = hp > 0.0 ? 1.0 : -1.0;
    // four independent partial sums (one per colour column c), so that the
    // FP64 multiply-add chains stay short
    double2 zc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) zc[c] = make_double2(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        double2 xu[4];  // X u_k
#pragma unroll
        for (int r = 0; r < 4; ++r)
            xu[r] = make_double2(fmadd(sg, X[r][k + 2].x, X[r][k].x), fmadd(sg, X[r][k + 2].y, X[r][k].y));
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double2 mx = make_double2(0.0, 0.0);  // (M^T X u_k)_c
#pragma unroll
            for (int r = 0; r < 4; ++r) cmac(mx, M[r][c], xu[r]);
            const double2 yu = make_double2(fmadd(sg, Y[k + 2][c].x, Y[k][c].x), fmadd(sg, Y[k + 2][c].y, Y[k][c].y));
            cmac(zc[c], yu, mx);
        }
    }
    const double2 z = make_double2((zc[0].x + zc[1].x) + (zc[2].x + zc[3].x), (zc[0].y + zc[1].y) + (zc[2].y + zc[3].y));
    return make_double2(0.5 * z.x, 0.5 * z.y);
}

// WD (Tr[P Y] <X, M> + Tr[P X] <Y, M>) + WE (<X P Y, M> + <Y P X, M>): the
// direct and the exchange terms with their weights (1, 1 for the proton).
template <int WD, int WE>
__device__ __forceinline__ double2 pair_term(const double2 X[4][4], const double2 Y[4][4], const double2 M[4][4],
                                            double hp) {
    double2 f = cmul(trace_p(Y, hp), inner_plain(X, M));
    cmac(f, trace_p(X, hp), inner_plain(Y, M));
    const double2 a = xpy_m(X, Y, M, hp);
    const double2 b = xpy_m(Y, X, M, hp);
    return make_double2(WD * f.x + WE * (a.x + b.x), WD * f.y + WE * (a.y + b.y));
}

// Kinds of baryon: the sink diquark matrix G (the source one follows) and
// the weights of the direct and exchange terms.  Delta++: with three
// identical quarks the six Wick terms pair up (the diquark tensors are
// antisymmetric under exchange of the two quarks they hold) into twice the
// direct and four times the exchange term of the proton form, with D = U,
// for each of G = C gamma_mu, mu = 1, 2, 3.  Every term is linear in
// M = G D G', so the sum over mu is taken on M: one colour sum with
// M = sum_mu G_mu D G'_mu.
template <int KIND, int MU>
struct BaryonKind {
    static constexpr SignedPerm G = KIND == QDP_BARYON_PROTON ? kCg5 : kCgamma[MU];
    static constexpr SignedPerm Gp = KIND == QDP_BARYON_PROTON ? sp_neg(kCg5) : source_diquark(kCgamma[MU]);
    static constexpr int WD = KIND == QDP_BARYON_PROTON ? 1 : 2;
    static constexpr int WE = KIND == QDP_BARYON_PROTON ? 1 : 4;
    static constexpr int NMU = KIND == QDP_BARYON_PROTON ? 1 : 3;
};

// M += G D G' with signed permutations (M = G D G' for the first mu, which
// writes every element: G' permutes the columns):
// M[r][G'.perm[q]] += i^(G.code[r] + G'.code[q]) D[G.perm[r]][q]
template <int KIND, int MU>
__device__ __forceinline__ void add_diquark(const double2 D[4][4], double2 M[4][4]) {
    using K = BaryonKind<KIND, MU>;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double2 z = times_ik(D[K::G.perm[r]][q], K::G.code[r] + K::Gp.code[q]);
            if constexpr (MU == 0) {
                M[r][K::Gp.perm[q]] = z;
            } else {
                M[r][K::Gp.perm[q]].x += z.x;
                M[r][K::Gp.perm[q]].y += z.y;
            }
        }
}

// One (b, b') colour step of the sum: s_b s_b' [ f(U^{xx'}, U^{yy'}) - f(U^{xy'}, U^{yx'}) ]
// (HALF = 1 or 2: only the first or only the second term, with its sign).
template <int PREC, bool BUF, int SRC, int B, int BP, int KIND, int HALF = 0>
__device__ __forceinline__ double2 colour_step(const BaryonArgs& A, int32_t s, const char* lane_rows, double hp) {
    using K = BaryonKind<KIND, 0>;
    constexpr int X0 = B == 0 ? 1 : 0, Y0 = B == 2 ? 1 : 2;
    constexpr int XP = BP == 0 ? 1 : 0, YP = BP == 2 ? 1 : 2;
    // (x, b, y) is an even permutation of (0, 1, 2) only for b = 1
    constexpr double SG = (B == 1 ? 1.0 : -1.0) * (BP == 1 ? 1.0 : -1.0);
    double2 M[4][4];
    {
        double2 D[4][4];
        get_block<PREC, BUF, SRC, true, B, BP>(A, s, lane_rows, D);
        add_diquark<KIND, 0>(D, M);
        if constexpr (K::NMU > 1) add_diquark<KIND, 1>(D, M);
        if constexpr (K::NMU > 2) add_diquark<KIND, 2>(D, M);
    }
    double2 X[4][4], Y[4][4];
    if constexpr (HALF == 1) {
        get_block<PREC, BUF, SRC, false, X0, XP>(A, s, lane_rows, X);
        get_block<PREC, BUF, SRC, false, Y0, YP>(A, s, lane_rows, Y);
        const double2 f1 = pair_term<K::WD, K::WE>(X, Y, M, hp);
        return make_double2(SG * f1.x, SG * f1.y);
    } else if constexpr (HALF == 2) {
        get_block<PREC, BUF, SRC, false, X0, YP>(A, s, lane_rows, X);
        get_block<PREC, BUF, SRC, false, Y0, XP>(A, s, lane_rows, Y);
        const double2 f2 = pair_term<K::WD, K::WE>(X, Y, M, hp);
        return make_double2(-SG * f2.x, -SG * f2.y);
    } else {
        get_block<PREC, BUF, SRC, false, X0, XP>(A, s, lane_rows, X);
        get_block<PREC, BUF, SRC, false, Y0, YP>(A, s, lane_rows, Y);
        const double2 f1 = pair_term<K::WD, K::WE>(X, Y, M, hp);
        get_block<PREC, BUF, SRC, false, X0, YP>(A, s, lane_rows, X);
        get_block<PREC, BUF, SRC, false, Y0, XP>(A, s, lane_rows, Y);
        const double2 f2 = pair_term<K::WD, K::WE>(X, Y, M, hp);
        return make_double2(SG * (f1.x - f2.x), SG * (f1.y - f2.y));
    }
}

template <int PREC, bool BUF, int SRC, int KIND, int HALF = 0>
__device__ __forceinline__ double2 colour_sum(const BaryonArgs& A, int32_t s, const char* lane_rows, double hp) {
    double2 acc = make_double2(0.0, 0.0);
    // the nine colour steps run one after another (a runtime loop, so the
    // compiler keeps one step's blocks live at a time)
#pragma unroll 1
    for (int bb = 0; bb < 9; ++bb) {
        double2 d;
        switch (__builtin_amdgcn_readfirstlane(bb)) {
            case 0: d = colour_step<PREC, BUF, SRC, 0, 0, KIND, HALF>(A, s, lane_rows, hp); break;
            case 1: d = colour_step<PREC, BUF, SRC, 0, 1, KIND, HALF>(A, s, lane_rows, hp); break;
            case 2: d = colour_step<PREC, BUF, SRC, 0, 2, KIND, HALF>(A, s, lane_rows, hp); break;
            case 3: d = colour_step<PREC, BUF, SRC, 1, 0, KIND, HALF>(A, s, lane_rows, hp); break;
            case 4: d = colour_step<PREC, BUF, SRC, 1, 1, KIND, HALF>(A, s, lane_rows, hp); break;
            case 5: d = colour_step<PREC, BUF, SRC, 1, 2, KIND, HALF>(A, s, lane_rows, hp); break;
            case 6: d = colour_step<PREC, BUF, SRC, 2, 0, KIND, HALF>(A, s, lane_rows, hp); break;
            case 7: d = colour_step<PREC, BUF, SRC, 2, 1, KIND, HALF>(A, s, lane_rows, hp); break;
            default: d = colour_step<PREC, BUF, SRC, 2, 2, KIND, HALF>(A, s, lane_rows, hp); break;
        }
        acc.x += d.x;
        acc.y += d.y;
    }
    return acc;
}

template <int PREC, bool BUF, int KIND>
__global__ __launch_bounds__(256) void baryon_kernel(BaryonArgs A) {
    const int t = blockIdx.y;
    const int chunk = blockIdx.x;
    const int64_t Vsh = A.g.Vsh;
    const int64_t Vs = 2 * Vsh;
    const double hp = 0.5 * A.parity;
    double2 acc = make_double2(0.0, 0.0);
    for (int64_t l = (int64_t)chunk * 256 + threadIdx.x; l < Vs; l += (int64_t)A.nchunks * 256) {
        const int64_t p = l >= Vsh ? 1 : 0;
        const int32_t s = (int32_t)(p * A.g.Vh + t * Vsh + (l - p * Vsh));
        const double2 d = colour_sum<PREC, BUF, 0, KIND>(A, s, nullptr, hp);
        acc.x += d.x;
        acc.y += d.y;
    }
    __shared__ double red[4][2];
    const double re = wave_sum(acc.x), im = wave_sum(acc.y);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w][0] = re;
        red[w][1] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double* out = A.partial + ((int64_t)t * A.nchunks + chunk) * 2;
        out[0] = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
        out[1] = (red[0][1] + red[1][1]) + (red[2][1] + red[3][1]);
    }
}

// F16S, buffer addressing: the same sums with the u propagator (and d, when
// SAME: d = u) staged in LDS per site, shared by a pair of wavefronts that
// take the two pair terms of every colour step (HALF 1: f(U^{xx'}, U^{yy'}),
// HALF 2: -f(U^{xy'}, U^{yx'})), so the 156 rows of 64 sites serve two
// wavefronts: a block of two pairs takes 78 KiB of LDS and two blocks fit a
// compute unit, two wavefronts per SIMD (rows per wavefront allowed one).
// Each wavefront copies half of the columns; the block's barriers order the
// copies and the reads.
template <int KIND, bool SAME>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void baryon_pair_kernel(BaryonArgs A) {
    __shared__ __attribute__((aligned(16))) char rows[2 * kBaryonLdsPairBytes];
    const int t = blockIdx.y;
    const int chunk = blockIdx.x;
    const int64_t Vsh = A.g.Vsh;
    const int64_t Vs = 2 * Vsh;
    const double hp = 0.5 * A.parity;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int pr = w >> 1, half = w & 1, lane = threadIdx.x & 63;
    char* prows = rows + pr * kBaryonLdsPairBytes;
    const char* lane_rows = prows + 4 * lane;
    double2 acc = make_double2(0.0, 0.0);
    for (int64_t base = (int64_t)chunk * 128; base < Vs; base += (int64_t)A.nchunks * 128) {
        const int64_t l = base + 64 * pr + lane;
        const bool active = l < Vs;
        const int64_t lc = active ? l : Vs - 1;
        const int64_t p = lc >= Vsh ? 1 : 0;
        const int32_t s = (int32_t)(p * A.g.Vh + t * Vsh + (lc - p * Vsh));
        __syncthreads();  // the previous sites' rows are no longer read
        stage_propagator_half_f16s(A.su, s, prows, half);
        wait_staged();
        __syncthreads();  // both halves of the rows have landed
        const double2 d = half ? colour_sum<QDP_F16S, true, SAME ? 2 : 1, KIND, 2>(A, s, lane_rows, hp)
                               : colour_sum<QDP_F16S, true, SAME ? 2 : 1, KIND, 1>(A, s, lane_rows, hp);
        if (active) {
            acc.x += d.x;
            acc.y += d.y;
        }
    }
    __syncthreads();
    double* red = reinterpret_cast<double*>(rows);
    const double re = wave_sum(acc.x), im = wave_sum(acc.y);
    if (lane == 0) {
        red[2 * w] = re;
        red[2 * w + 1] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double* out = A.partial + ((int64_t)t * A.nchunks + chunk) * 2;
        out[0] = (red[0] + red[2]) + (red[4] + red[6]);
        out[1] = (red[1] + red[3]) + (red[5] + red[7]);
    }
}

// out[(t - t0 mod Lt) * 2 + k] = sum over chunks, fixed order.
__global__ void baryon_finish(const double* __restrict__ partial, int32_t Lt, int32_t nchunks, int32_t t0,
                               double* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Lt) return;
    double re = 0.0, im = 0.0;
    for (int c = 0; c < nchunks; ++c) {
        re += partial[((int64_t)t * nchunks + c) * 2];
        im += partial[((int64_t)t * nchunks + c) * 2 + 1];
    }
    const int tr = ((t - t0) % Lt + Lt) % Lt;
    out[2 * tr] = re;
    out[2 * tr + 1] = im;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------


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
constexpr int kMomPerLaunch = 4;

template <bool BUF, int NMOM>
void* meson_func_buf(int prec) {
    switch (prec) {
        case QDP_F64: return reinterpret_cast<void*>(&meson_kernel<QDP_F64, BUF, NMOM>);
        case QDP_F32: return reinterpret_cast<void*>(&meson_kernel<QDP_F32, BUF, NMOM>);
        default: return reinterpret_cast<void*>(&meson_kernel<QDP_F16S, BUF, NMOM>);
    }
}

void* meson_func(int prec, bool buf, bool mom) {
    if (mom) return buf ? meson_func_buf<true, kMomPerLaunch>(prec) : meson_func_buf<false, kMomPerLaunch>(prec);
    return buf ? meson_func_buf<true, 0>(prec) : meson_func_buf<false, 0>(prec);
}

// F16S contractions run the one-wavefront-per-colour kernels (with momenta:
// when S1 and S2 are the same columns; two propagators' registers and the
// momentum sums do not fit one wavefront's registers)
bool meson_by_colour(int prec, bool mom, bool alias) { return prec == QDP_F16S && (!mom || alias); }
static_assert(kColourMomenta == kMomPerLaunch, "one wavefront per momentum of a launch");
void* meson_colour_func(bool buf, bool alias, bool mom) {
    if (mom) return buf ? reinterpret_cast<void*>(&meson_colour_mom_kernel<true, true>)
                        : reinterpret_cast<void*>(&meson_colour_mom_kernel<false, true>);
    if (buf) return alias ? reinterpret_cast<void*>(&meson_colour_kernel<true, true>)
                          : reinterpret_cast<void*>(&meson_colour_kernel<true, false>);
    return alias ? reinterpret_cast<void*>(&meson_colour_kernel<false, true>)
                 : reinterpret_cast<void*>(&meson_colour_kernel<false, false>);
}
}  // namespace

namespace {
// Checks the 24 column handles, pins the columns (resident_only: fail
// instead of filling a column from host memory) and fills the kernel
// arguments shared by the contraction entry points.
qdp_status meson_setup(Ctx* ctx, const uint64_t* S1, const uint64_t* S2, int32_t j_decay, bool resident_only,
                       PinSet& pins, ContractArgs* a, int32_t* prec_out) {
    if (j_decay != 3) return set_error(ctx, QDP_ERR_UNSUPPORTED, "contract: only j_decay = 3 (time)");
    uint64_t lat = 0;
    int32_t prec = -1;
    for (int side = 0; side < 2; ++side)
        for (int c = 0; c < 12; ++c) {
            const uint64_t id = side ? S2[c] : S1[c];
            Field* f = find_field(ctx, id);
            if (!f) return set_error(ctx, QDP_ERR_STATE, "contract: unknown column handle");
            if (f->type != QDP_FERMION) return set_error(ctx, QDP_ERR_TYPE, "contract: columns must be FERMION");
            if (lat && f->lattice != lat) return set_error(ctx, QDP_ERR_LATTICE, "contract: columns on different lattices");
            if (prec >= 0 && f->prec != prec)
                return set_error(ctx, QDP_ERR_UNSUPPORTED, "contract: all 24 columns must share one precision");
            if (resident_only) {
                const CacheEntry* e = ctx->cache.find(id);
                if (!e || !e->on_device)
                    return set_error(ctx, QDP_ERR_STATE,
                                     "contract: column %llu is spilled to host memory; this call does not refill it",
                                     (unsigned long long)id);
            }
            lat = f->lattice;
            prec = f->prec;
        }
    const Geometry g = find_lattice(ctx, lat)->geo;
    const int32_t Lt = g.L[3];
    const int64_t Vs = 2 * g.Vsh;
    int64_t nchunks = (8192 + Lt - 1) / Lt;
    nchunks = std::max<int64_t>(1, std::min<int64_t>(nchunks, (Vs + 63) / 64));

    *a = ContractArgs{};
    a->g = g;
    for (int c = 0; c < 12; ++c) {
        char* p;
        QDP_CHECK(pins.add(S1[c], true, &p));
        a->s1[c] = p;
        QDP_CHECK(pins.add(S2[c], true, &p));
        a->s2[c] = p;
    }
    a->nchunks = (int32_t)nchunks;
    *prec_out = prec;
    return QDP_OK;
}

// Bytes of the per-block partial sums of one meson launch carrying nq momenta.
size_t meson_partial_bytes(const ContractArgs& a, int32_t nq) {
    return sizeof(double) * 2 * 16 * (size_t)nq * a.g.L[3] * (size_t)a.nchunks;
}

// One meson launch (a.partial set, a.mom the launch's momenta) and its
// fixed-order finish into d_out: nq * 16 * Lt complex values.
qdp_status meson_launch(Ctx* ctx, ContractArgs& a, int32_t prec, bool mom, uint32_t mask, int32_t t0,
                        double* d_out) {
    const int32_t Lt = a.g.L[3];
    const int32_t nq = mom ? kMomPerLaunch : 1;
    void* args[] = {&a};
    const bool buf = field_bytes(a.g, QDP_FERMION, prec) < (int64_t(1) << 32) && !(ctx->flags & QDP_INIT_FLAT_ADDRESSING);
    bool alias = true;
    for (int c = 0; c < 12; ++c) alias = alias && a.s1[c] == a.s2[c];
    if (meson_by_colour(prec, mom, alias)) {
        QDP_HIP(ctx, hipLaunchKernel(meson_colour_func(buf, alias, mom), dim3((unsigned)a.nchunks, (unsigned)Lt),
                                     dim3(mom ? 256 : 192), args, 0, ctx->stream));
    } else {
        QDP_HIP(ctx, hipLaunchKernel(meson_func(prec, buf, mom), dim3((unsigned)a.nchunks, (unsigned)Lt),
                                     dim3(256), args, 0, ctx->stream));
    }
    QDP_CHECK(check_launch(ctx, "meson kernel"));
    const int nthreads = nq * 16 * Lt;
    hipLaunchKernelGGL(meson_finish, dim3((nthreads + 255) / 256), dim3(256), 0, ctx->stream, a.partial, Lt,
                       a.nchunks, nq, mask, t0, d_out);
    return check_launch(ctx, "meson finish kernel");
}
}  // namespace

qdp_status hadron_contract_impl(Ctx* ctx, const uint64_t* S1, const uint64_t* S2, uint32_t mask,
                                int32_t t0, int32_t j_decay, const int32_t* moms, int32_t nmom, double* out) {
    if (nmom < 0 || (nmom > 0 && !moms)) return set_error(ctx, QDP_ERR_ARG, "contract: bad momentum list");
    PinSet pins(ctx);
    ContractArgs a;
    int32_t prec;
    QDP_CHECK(meson_setup(ctx, S1, S2, j_decay, false, pins, &a, &prec));
    const int32_t Lt = a.g.L[3];
    const bool mom = nmom > 0;
    const int32_t nq = mom ? kMomPerLaunch : 1;  // momenta per launch
    const int32_t nlaunch = mom ? (nmom + kMomPerLaunch - 1) / kMomPerLaunch : 1;
    PoolTemp scratch;
    const size_t partial_bytes = meson_partial_bytes(a, nq);
    const size_t launch_out_bytes = sizeof(double) * 2 * 16 * (size_t)nq * Lt;
    const size_t out_bytes = sizeof(double) * 2 * 16 * (size_t)Lt * (mom ? nmom : 1);
    QDP_CHECK(scratch.alloc(ctx, (int64_t)(partial_bytes + launch_out_bytes * nlaunch + 256)));
    a.partial = reinterpret_cast<double*>(scratch.ptr());
    double* d_out = reinterpret_cast<double*>(scratch.ptr() + ((partial_bytes + 255) & ~size_t(255)));

    for (int32_t L = 0; L < nlaunch; ++L) {
        for (int q = 0; q < kMomPerLaunch; ++q)
            for (int i = 0; i < 3; ++i) {
                const int32_t k = L * kMomPerLaunch + q;
                a.mom[q][i] = (mom && k < nmom) ? moms[3 * k + i] : 0;
            }
        QDP_CHECK(meson_launch(ctx, a, prec, mom, mask, t0, d_out + (size_t)L * nq * 16 * Lt * 2));
    }
    double* host;
    QDP_CHECK(host_result_buffer(ctx, out_bytes, &host));
    QDP_HIP(ctx, hipMemcpyAsync(host, d_out, out_bytes, hipMemcpyDeviceToHost, ctx->stream));
    QDP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::memcpy(out, host, out_bytes);
    return QDP_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free zero-momentum contraction: the per-block partial sums live
// in a fixed device array of the library instead of a pool temporary.  The
// array is one per GPU; its device address is looked up once per device
// when a context is created there (in host code the array's name is not a
// device address).  Calls on one GPU share it, so calls that overlap in time
// on one GPU (two streams or two contexts) race; every call writes all of
// the partial sums it reads, so nothing needs clearing between calls.
// ---------------------------------------------------------------------------

constexpr size_t kNoAllocScratchBytes = size_t(4) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};
}  // namespace

qdp_status noalloc_scratch_init(Ctx* ctx) {
    if (ctx->device < 0 || ctx->device >= kMaxDevices)
        return set_error(ctx, QDP_ERR_ARG, "device index %d out of range", ctx->device);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[ctx->device]) {
        void* p = nullptr;
        // the calling thread has ctx->device current (qdp_init set it)
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_error(ctx, e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                    "hipGetSymbolAddress(scratch)");
        g_scratch_dev[ctx->device] = p;
    }
    ctx->noalloc_scratch = g_scratch_dev[ctx->device];
    return QDP_OK;
}

qdp_status hadron_contract_noalloc_impl(Ctx* ctx, const uint64_t* S1, const uint64_t* S2, uint32_t mask,
                                        int32_t t0, int32_t j_decay, double* out_dev) {
    if (!out_dev) return set_error(ctx, QDP_ERR_ARG, "contract_noalloc: null output");
    if (reinterpret_cast<uintptr_t>(out_dev) % alignof(double))
        return set_error(ctx, QDP_ERR_ARG, "contract_noalloc: output not 8-byte aligned");
    if (!ctx->noalloc_scratch) return set_error(ctx, QDP_ERR_STATE, "contract_noalloc: scratch array not set up");
    PinSet pins(ctx);
    ContractArgs a;
    int32_t prec;
    QDP_CHECK(meson_setup(ctx, S1, S2, j_decay, true, pins, &a, &prec));
    const size_t partial_bytes = meson_partial_bytes(a, 1);
    if (partial_bytes > kNoAllocScratchBytes)
        return set_error(ctx, QDP_ERR_UNSUPPORTED,
                         "contract_noalloc: %zu bytes of partial sums (Lt %d) exceed the %zu-byte scratch array",
                         partial_bytes, a.g.L[3], kNoAllocScratchBytes);
    a.partial = static_cast<double*>(ctx->noalloc_scratch);
    return meson_launch(ctx, a, prec, false, mask, t0, out_dev);
}

namespace {
template <bool BUF, int KIND>
void* baryon_func_kind(int prec) {
    switch (prec) {
        case QDP_F64: return reinterpret_cast<void*>(&baryon_kernel<QDP_F64, BUF, KIND>);
        case QDP_F32: return reinterpret_cast<void*>(&baryon_kernel<QDP_F32, BUF, KIND>);
        default:
            // F16S with buffer addressing runs baryon_pair_kernel
            if constexpr (BUF) return nullptr;
            else return reinterpret_cast<void*>(&baryon_kernel<QDP_F16S, false, KIND>);
    }
}
// F16S with buffer addressing stages the propagator in LDS for wavefront
// pairs (both propagators when the u and d columns are the same fields).
void* baryon_func(int prec, bool buf, int kind, bool same) {
    if (prec == QDP_F16S && buf) {
        if (kind == QDP_BARYON_PROTON)
            return same ? reinterpret_cast<void*>(&baryon_pair_kernel<QDP_BARYON_PROTON, true>)
                        : reinterpret_cast<void*>(&baryon_pair_kernel<QDP_BARYON_PROTON, false>);
        return reinterpret_cast<void*>(&baryon_pair_kernel<QDP_BARYON_DELTA_PP, true>);
    }
    if (kind == QDP_BARYON_PROTON) return buf ? baryon_func_kind<true, QDP_BARYON_PROTON>(prec)
                                              : baryon_func_kind<false, QDP_BARYON_PROTON>(prec);
    return buf ? baryon_func_kind<true, QDP_BARYON_DELTA_PP>(prec) : baryon_func_kind<false, QDP_BARYON_DELTA_PP>(prec);
}
}  // namespace

qdp_status baryon_contract_impl(Ctx* ctx, const uint64_t* Su, const uint64_t* Sd, int32_t kind, int32_t parity,
                                int32_t t0, int32_t j_decay, double* out) {
    if (j_decay != 3) return set_error(ctx, QDP_ERR_UNSUPPORTED, "baryon: only j_decay = 3 (time)");
    if (kind != QDP_BARYON_PROTON && kind != QDP_BARYON_DELTA_PP)
        return set_error(ctx, QDP_ERR_UNSUPPORTED, "baryon: unknown kind %d", kind);
    if (kind == QDP_BARYON_DELTA_PP) Sd = Su;  // three u quarks: one propagator
    if (parity != 1 && parity != -1) return set_error(ctx, QDP_ERR_ARG, "baryon: parity must be +1 or -1");
    uint64_t lat = 0;
    int32_t prec = -1;
    for (int side = 0; side < 2; ++side)
        for (int c = 0; c < 12; ++c) {
            Field* f = find_field(ctx, side ? Sd[c] : Su[c]);
            if (!f) return set_error(ctx, QDP_ERR_STATE, "baryon: unknown column handle");
            if (f->type != QDP_FERMION) return set_error(ctx, QDP_ERR_TYPE, "baryon: columns must be FERMION");
            if (lat && f->lattice != lat) return set_error(ctx, QDP_ERR_LATTICE, "baryon: columns on different lattices");
            if (prec >= 0 && f->prec != prec)
                return set_error(ctx, QDP_ERR_UNSUPPORTED, "baryon: all 24 columns must share one precision");
            lat = f->lattice;
            prec = f->prec;
        }
    const Geometry g = find_lattice(ctx, lat)->geo;
    const int32_t Lt = g.L[3];
    const int64_t Vs = 2 * g.Vsh;
    int64_t nchunks = (8192 + Lt - 1) / Lt;
    nchunks = std::max<int64_t>(1, std::min<int64_t>(nchunks, (Vs + 255) / 256));

    PinSet pins(ctx);
    BaryonArgs a{};
    a.g = g;
    for (int c = 0; c < 12; ++c) {
        char* p;
        QDP_CHECK(pins.add(Su[c], true, &p));
        a.su[c] = p;
        QDP_CHECK(pins.add(Sd[c], true, &p));
        a.sd[c] = p;
    }
    a.nchunks = (int32_t)nchunks;
    a.parity = parity;

    PoolTemp scratch;
    const size_t partial_bytes = sizeof(double) * 2 * (size_t)Lt * nchunks;
    const size_t out_bytes = sizeof(double) * 2 * (size_t)Lt;
    QDP_CHECK(scratch.alloc(ctx, (int64_t)(partial_bytes + out_bytes + 256)));
    a.partial = reinterpret_cast<double*>(scratch.ptr());
    double* d_out = reinterpret_cast<double*>(scratch.ptr() + ((partial_bytes + 255) & ~size_t(255)));
    void* args[] = {&a};
    const bool buf = field_bytes(g, QDP_FERMION, prec) < (int64_t(1) << 32) && !(ctx->flags & QDP_INIT_FLAT_ADDRESSING);
    bool same = true;
    for (int c = 0; c < 12; ++c) same = same && a.su[c] == a.sd[c];
    QDP_HIP(ctx, hipLaunchKernel(baryon_func(prec, buf, kind, same), dim3((unsigned)nchunks, (unsigned)Lt),
                                 dim3(256), args, 0, ctx->stream));
    QDP_CHECK(check_launch(ctx, "baryon kernel"));
    hipLaunchKernelGGL(baryon_finish, dim3((Lt + 255) / 256), dim3(256), 0, ctx->stream, a.partial, Lt,
                       (int32_t)nchunks, t0, d_out);
    QDP_CHECK(check_launch(ctx, "baryon finish kernel"));
    double* host;
    QDP_CHECK(host_result_buffer(ctx, out_bytes, &host));
    QDP_HIP(ctx, hipMemcpyAsync(host, d_out, out_bytes, hipMemcpyDeviceToHost, ctx->stream));
    QDP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::memcpy(out, host, out_bytes);
    return QDP_OK;
}

}  // namespace qdpmi
