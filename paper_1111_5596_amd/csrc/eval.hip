// Expression lowering: qdp_eval, qdp_shift and qdp_sum_multi.
//
// The paper builds each expression's tree at compile time (PETE), emits GPU
// code for it and JIT-compiles it (section 4.2, Figure 3).  Here the tree
// arrives at run time as a postfix program and is lowered onto kernels that
// were compiled ahead of time for gfx950:
//   1. parse and type-check (QDP++ product rules: spin parts and colour
//      parts multiply as matrices, a scalar part acts as the identity);
//   2. push every shift down to the leaves, shift(f(a, b)) = f(shift a,
//      shift b) for site-local f, so that a leaf carries a displacement and
//      no intermediate value ever needs its neighbours;
//   3. match the tree against a fused kernel: sums of c_k [adj] M_k(x+d_k)
//      V_k(x+e_k) and c_k V_k(x+e_k) with M a colour matrix and V a fermion
//      or colour vector (axpy, U psi, U^dagger psi with shifts, the whole
//      Jacobi step) run as one pass;
//   4. otherwise evaluate node by node: one kernel per internal node,
//      instantiated per (operation, operand types, FP32 / FP64), reading
//      leaves straight from their fields and intermediates from pool
//      temporaries.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <utility>
#include <vector>

#include "device.hpp"
#include "internal.hpp"

namespace qdpmi {

// ---------------------------------------------------------------------------
// Type rules (host and device)
// ---------------------------------------------------------------------------

enum NodeOp : int32_t {
    K_NEG = 0, K_CONJ, K_ADJ, K_TRACE, K_TRACE_COLOR, K_TRACE_SPIN, K_REAL, K_IMAG, K_NORM2,
    K_GAMMA_L, K_GAMMA_R, K_COPY,  // unary
    K_ADD, K_SUB, K_MUL, K_INNER,  // binary
    K_TRACE_MUL,                   // binary, formed by the lowering: trace(a b)
    K_NUM_OPS
};
constexpr int kNumTypes = 7;  // REAL .. PROPAGATOR

struct Shp {
    int s1, s2, c1, c2;
};

constexpr Shp shp(int t) {
    return t == QDP_REAL || t == QDP_COMPLEX ? Shp{1, 1, 1, 1}
         : t == QDP_COLOR_VECTOR            ? Shp{1, 1, 3, 1}
         : t == QDP_COLOR_MATRIX            ? Shp{1, 1, 3, 3}
         : t == QDP_FERMION                 ? Shp{4, 1, 3, 1}
         : t == QDP_SPIN_MATRIX             ? Shp{4, 4, 1, 1}
                                            : Shp{4, 4, 3, 3};
}
constexpr int ncomp_of(int t) { return shp(t).s1 * shp(t).s2 * shp(t).c1 * shp(t).c2; }
constexpr bool is_scalar(int t) { return t == QDP_REAL || t == QDP_COMPLEX; }

constexpr int type_of_shape(Shp s, bool real) {
    return (s.s1 == 1 && s.s2 == 1 && s.c1 == 1 && s.c2 == 1) ? (real ? QDP_REAL : QDP_COMPLEX)
         : (s.s1 == 1 && s.s2 == 1 && s.c1 == 3 && s.c2 == 1) ? QDP_COLOR_VECTOR
         : (s.s1 == 1 && s.s2 == 1 && s.c1 == 3 && s.c2 == 3) ? QDP_COLOR_MATRIX
         : (s.s1 == 4 && s.s2 == 1 && s.c1 == 3 && s.c2 == 1) ? QDP_FERMION
         : (s.s1 == 4 && s.s2 == 4 && s.c1 == 1 && s.c2 == 1) ? QDP_SPIN_MATRIX
         : (s.s1 == 4 && s.s2 == 4 && s.c1 == 3 && s.c2 == 3) ? QDP_PROPAGATOR
                                                               : -1;
}

// Product of two (row, col) factor shapes; {-1,-1} if not multipliable.
struct Pair {
    int r, c;
};
constexpr Pair mul_part(int ar, int ac, int br, int bc) {
    return (ar == 1 && ac == 1) ? Pair{br, bc}
         : (br == 1 && bc == 1) ? Pair{ar, ac}
         : (ac == br)           ? Pair{ar, bc}
                                : Pair{-1, -1};
}

constexpr int mul_type(int a, int b) {
    return (mul_part(shp(a).s1, shp(a).s2, shp(b).s1, shp(b).s2).r < 0 ||
            mul_part(shp(a).c1, shp(a).c2, shp(b).c1, shp(b).c2).r < 0)
               ? -1
               : type_of_shape(Shp{mul_part(shp(a).s1, shp(a).s2, shp(b).s1, shp(b).s2).r,
                                   mul_part(shp(a).s1, shp(a).s2, shp(b).s1, shp(b).s2).c,
                                   mul_part(shp(a).c1, shp(a).c2, shp(b).c1, shp(b).c2).r,
                                   mul_part(shp(a).c1, shp(a).c2, shp(b).c1, shp(b).c2).c},
                               a == QDP_REAL && b == QDP_REAL);
}

// Result type of (op, a, b), -1 when invalid.
constexpr int result_type(int op, int a, int b) {
    return op == K_NEG || op == K_CONJ || op == K_COPY ? a
         : op == K_ADJ    ? ((shp(a).s1 == shp(a).s2 && shp(a).c1 == shp(a).c2) ? a : -1)
         : op == K_TRACE  ? (a == QDP_REAL ? QDP_REAL
                             : (a == QDP_COMPLEX || a == QDP_COLOR_MATRIX || a == QDP_SPIN_MATRIX ||
                                a == QDP_PROPAGATOR) ? QDP_COMPLEX : -1)
         : op == K_TRACE_COLOR ? (a == QDP_COLOR_MATRIX ? QDP_COMPLEX : a == QDP_PROPAGATOR ? QDP_SPIN_MATRIX : -1)
         : op == K_TRACE_SPIN  ? (a == QDP_SPIN_MATRIX ? QDP_COMPLEX : a == QDP_PROPAGATOR ? QDP_COLOR_MATRIX : -1)
         : op == K_REAL || op == K_IMAG ? (is_scalar(a) ? QDP_REAL : -1)
         : op == K_NORM2   ? QDP_REAL
         : op == K_GAMMA_L ? (shp(a).s1 == 4 ? a : -1)
         : op == K_GAMMA_R ? (shp(a).s2 == 4 ? a : -1)
         : op == K_ADD || op == K_SUB ? (a == b ? a : (is_scalar(a) && is_scalar(b)) ? QDP_COMPLEX : -1)
         : op == K_MUL   ? mul_type(a, b)
         : op == K_INNER ? (a == b ? QDP_COMPLEX : -1)
         : op == K_TRACE_MUL ? ((a == b && (a == QDP_COLOR_MATRIX || a == QDP_SPIN_MATRIX || a == QDP_PROPAGATOR))
                                    ? QDP_COMPLEX : -1)
                         : -1;
}

constexpr bool is_binary(int op) { return op >= K_ADD; }

// ---------------------------------------------------------------------------
// Device-side operand access
// ---------------------------------------------------------------------------

enum { OPND_FIELD = 0, OPND_CONST = 1 };

struct Operand {
    const char* base;
    int32_t kind, prec, rec, nrec, ncomp;
    int32_t d[4];
    int32_t has_disp;
    int32_t pad;
    double cre, cim;
};

struct SubsetDesc {
    int32_t kind;  // qdp_subset_kind
    int32_t t;
    int64_t count;
};

struct OutDesc {
    char* base;
    int32_t prec, nrec, ncomp, real_only;
};

struct GammaTab {
    int8_t perm[16][4];
    int8_t code[16][4];
};

__device__ __forceinline__ int64_t subset_site(const Geometry& g, const SubsetDesc& sub, int64_t l) {
    switch (sub.kind) {
        case QDP_ODD: return g.Vh + l;
        case QDP_TIMESLICE: {
            const int64_t p = l >= g.Vsh ? 1 : 0;
            return p * g.Vh + (int64_t)sub.t * g.Vsh + (l - p * g.Vsh);
        }
        default: return l;  // ALL, EVEN
    }
}

__device__ __forceinline__ int32_t displaced_site(const Geometry& g, const int32_t c[4], const int32_t d[4]) {
    int32_t y[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        int32_t v = (c[mu] + d[mu]) % g.L[mu];
        y[mu] = v < 0 ? v + g.L[mu] : v;
    }
    return (int32_t)cb_index(g, y[0], y[1], y[2], y[3]);
}

template <typename R>
__device__ __forceinline__ cplx_t<R> load_comp(const char* base, int32_t prec, int32_t nrec, int32_t ncomp,
                                               int32_t rec, int32_t k, int32_t site) {
    using T2 = cplx_t<R>;
    const char* p = base + comp_offset(nrec, ncomp, prec, rec, k, site);
    if (prec == QDP_F64) {
        const double2 v = *reinterpret_cast<const double2*>(p);
        return T2{(R)v.x, (R)v.y};
    } else if (prec == QDP_F32) {
        const float2 v = *reinterpret_cast<const float2*>(p);
        return T2{(R)v.x, (R)v.y};
    } else {
        const half2_t h = *reinterpret_cast<const half2_t*>(p);
        const float sc = *reinterpret_cast<const float*>(base + scale_offset(nrec, ncomp, rec, site));
        return T2{(R)((float)h.x * sc), (R)((float)h.y * sc)};
    }
}

// N consecutive components of a chunked F32 or F16S field whose first one
// sits at position OFF of its 16-byte chunk (p: that chunk at this site):
// every chunk the run touches is loaded once, whole (the partly used first
// and last chunks lie inside the site's record rows).
template <typename R, typename E, int OFF, int N>
__device__ __forceinline__ void load_run(const char* p, float sc, cplx_t<R>* v) {
    constexpr int CE = 16 / (int)sizeof(E);
    constexpr int NCH = (OFF + N + CE - 1) / CE;
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
        const Chunk<E> w = __builtin_bit_cast(Chunk<E>, *reinterpret_cast<const u32x4_t*>(p + q * 1024));
#pragma unroll
        for (int j = 0; j < CE; ++j) {
            const int k = q * CE + j - OFF;
            if (k >= 0 && k < N) {
                if constexpr (sizeof(E) == 4) v[k] = cplx_t<R>{(R)((float)w.v[j].x * sc), (R)((float)w.v[j].y * sc)};
                else v[k] = cplx_t<R>{(R)w.v[j].x, (R)w.v[j].y};
            }
        }
    }
}

// N consecutive components of record rec (from component 0): whole 16-byte
// chunks when the field is chunked (F32: 2 components per load, F16S: 4;
// short runs such as a link of the gauge field from any position in its
// chunk), else one component at a time.
template <typename R, int N>
__device__ __forceinline__ void load_comps(const char* base, int32_t prec, int32_t nrec, int32_t ncomp, int32_t rec,
                                           int32_t site, cplx_t<R>* v) {
    using T2 = cplx_t<R>;
    const int32_t e0 = rec * ncomp;
    if constexpr (N <= 16) {
        if (prec != QDP_F64 && chunked_layout(nrec, ncomp, prec)) {
            // the chunk holding element e0
            const int32_t les = prec_log2_bytes(prec), pos = e0 & ((1 << (4 - les)) - 1);
            const char* p = base + comp_offset(nrec, ncomp, prec, rec, 0, site) - (pos << les);
            if (prec == QDP_F32) {
                if (pos == 0) load_run<R, float2, 0, N>(p, 1.f, v);
                else load_run<R, float2, 1, N>(p, 1.f, v);
            } else {
                const float sc = *reinterpret_cast<const float*>(base + scale_offset(nrec, ncomp, rec, site));
                switch (pos) {
                    case 0: load_run<R, half2_t, 0, N>(p, sc, v); break;
                    case 1: load_run<R, half2_t, 1, N>(p, sc, v); break;
                    case 2: load_run<R, half2_t, 2, N>(p, sc, v); break;
                    default: load_run<R, half2_t, 3, N>(p, sc, v); break;
                }
            }
            return;
        }
    }
    if constexpr (N % 2 == 0) {
        if (prec == QDP_F32 && chunked_layout(nrec, ncomp, prec) && e0 % 2 == 0) {
            const char* p = base + comp_offset(nrec, ncomp, prec, rec, 0, site);
#pragma unroll
            for (int q = 0; q < N / 2; ++q) {
                const float4 w = *reinterpret_cast<const float4*>(p + q * 1024);
                v[2 * q] = T2{(R)w.x, (R)w.y};
                v[2 * q + 1] = T2{(R)w.z, (R)w.w};
            }
            return;
        }
    }
    if constexpr (N % 4 == 0) {
        if (prec == QDP_F16S && chunked_layout(nrec, ncomp, prec) && e0 % 4 == 0) {
            const char* p = base + comp_offset(nrec, ncomp, prec, rec, 0, site);
            const float sc = *reinterpret_cast<const float*>(base + scale_offset(nrec, ncomp, rec, site));
#pragma unroll
            for (int q = 0; q < N / 4; ++q) {
                const Chunk<half2_t> w = __builtin_bit_cast(Chunk<half2_t>, *reinterpret_cast<const u32x4_t*>(p + q * 1024));
#pragma unroll
                for (int j = 0; j < 4; ++j) v[4 * q + j] = T2{(R)((float)w.v[j].x * sc), (R)((float)w.v[j].y * sc)};
            }
            return;
        }
    }
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = load_comp<R>(base, prec, nrec, ncomp, rec, k, site);
}

template <int T, typename R>
__device__ __forceinline__ void load_operand(const Operand& op, const Geometry& g, int32_t s,
                                             const int32_t c[4], cplx_t<R>* v) {
    constexpr int N = ncomp_of(T);
    if (op.kind == OPND_CONST) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = cplx_t<R>{(R)op.cre, (R)op.cim};
        return;
    }
    const int32_t site = op.has_disp ? displaced_site(g, c, op.d) : s;
    load_comps<R, N>(op.base, op.prec, op.nrec, op.ncomp, op.rec, site, v);
}

template <typename R>
__device__ __forceinline__ void store_values(const OutDesc& out, const Geometry& g, int32_t s,
                                             const cplx_t<R>* v, int N) {
    if (out.prec == QDP_F64) {
        for (int k = 0; k < N; ++k) {
            double2 w = make_double2((double)v[k].x, out.real_only ? 0.0 : (double)v[k].y);
            *reinterpret_cast<double2*>(out.base + comp_offset(out.nrec, out.ncomp, out.prec, 0, k, s)) = w;
        }
    } else if (out.prec == QDP_F32) {
        if (N % 2 == 0 && chunked_layout(out.nrec, out.ncomp, out.prec)) {
            // whole 16-byte chunks (the output record starts the site's chunks)
            char* p = out.base + comp_offset(out.nrec, out.ncomp, out.prec, 0, 0, s);
            for (int q = 0; q < N / 2; ++q)
                *reinterpret_cast<float4*>(p + q * 1024) =
                    make_float4((float)v[2 * q].x, out.real_only ? 0.f : (float)v[2 * q].y, (float)v[2 * q + 1].x,
                                out.real_only ? 0.f : (float)v[2 * q + 1].y);
            return;
        }
        for (int k = 0; k < N; ++k) {
            float2 w = make_float2((float)v[k].x, out.real_only ? 0.f : (float)v[k].y);
            *reinterpret_cast<float2*>(out.base + comp_offset(out.nrec, out.ncomp, out.prec, 0, k, s)) = w;
        }
    } else {
        float m = 0.f;
        for (int k = 0; k < N; ++k) {
            m = fmaxf(m, fabsf((float)v[k].x));
            if (!out.real_only) m = fmaxf(m, fabsf((float)v[k].y));
        }
        const int e = f16s_exponent(m);
        for (int k = 0; k < N; ++k)
            *reinterpret_cast<half2_t*>(out.base + comp_offset(out.nrec, out.ncomp, out.prec, 0, k, s)) =
                f16s_encode((float)v[k].x, out.real_only ? 0.f : (float)v[k].y, e);
        *reinterpret_cast<float*>(out.base + scale_offset(out.nrec, out.ncomp, 0, s)) =
            f16s_scale(m, e);
    }
}

// ---------------------------------------------------------------------------
// Per-node kernels
// ---------------------------------------------------------------------------

struct NodeArgs {
    Geometry g;
    SubsetDesc sub;
    Operand a, b;
    OutDesc out;
    GammaTab gt;
    int32_t gamma_n;
    int32_t need_coords;
};

template <int S1, int S2, int C1, int C2>
struct Idx {
    static constexpr int at(int i, int k, int x, int z) { return ((i * S2 + k) * C1 + x) * C2 + z; }
};

template <typename T2>
__device__ __forceinline__ T2 cmul(const T2& a, const T2& b) {
    T2 r;
    r.x = fmadd(a.x, b.x, -(a.y * b.y));
    r.y = fmadd(a.x, b.y, a.y * b.x);
    return r;
}

template <typename T2>
__device__ __forceinline__ T2 phase(int code, const T2& z) {
    switch (code & 3) {
        case 0: return z;
        case 1: return T2{-z.y, z.x};
        case 2: return T2{-z.x, -z.y};
        default: return T2{z.y, -z.x};
    }
}

template <int OP, int TA, int TB, typename R>
__device__ __forceinline__ void apply_op(const NodeArgs& A, const cplx_t<R>* a, const cplx_t<R>* b, cplx_t<R>* r) {
    using T2 = cplx_t<R>;
    constexpr Shp sa = shp(TA), sb = shp(TB);
    constexpr int NA = ncomp_of(TA);
    if constexpr (OP == K_NEG) {
        for (int k = 0; k < NA; ++k) r[k] = T2{-a[k].x, -a[k].y};
    } else if constexpr (OP == K_CONJ) {
        for (int k = 0; k < NA; ++k) r[k] = T2{a[k].x, -a[k].y};
    } else if constexpr (OP == K_COPY) {
        for (int k = 0; k < NA; ++k) r[k] = a[k];
    } else if constexpr (OP == K_ADJ) {
        using I = Idx<sa.s1, sa.s2, sa.c1, sa.c2>;
        for (int i = 0; i < sa.s1; ++i)
            for (int k = 0; k < sa.s2; ++k)
                for (int x = 0; x < sa.c1; ++x)
                    for (int z = 0; z < sa.c2; ++z) {
                        const T2 v = a[I::at(k, i, z, x)];
                        r[I::at(i, k, x, z)] = T2{v.x, -v.y};
                    }
    } else if constexpr (OP == K_TRACE) {
        using I = Idx<sa.s1, sa.s2, sa.c1, sa.c2>;
        T2 acc{0, 0};
        for (int i = 0; i < sa.s1; ++i)
            for (int x = 0; x < sa.c1; ++x) {
                acc.x += a[I::at(i, i, x, x)].x;
                acc.y += a[I::at(i, i, x, x)].y;
            }
        r[0] = acc;
    } else if constexpr (OP == K_TRACE_COLOR) {
        using I = Idx<sa.s1, sa.s2, sa.c1, sa.c2>;
        for (int i = 0; i < sa.s1; ++i)
            for (int k = 0; k < sa.s2; ++k) {
                T2 acc{0, 0};
                for (int x = 0; x < sa.c1; ++x) {
                    acc.x += a[I::at(i, k, x, x)].x;
                    acc.y += a[I::at(i, k, x, x)].y;
                }
                r[i * sa.s2 + k] = acc;
            }
    } else if constexpr (OP == K_TRACE_SPIN) {
        using I = Idx<sa.s1, sa.s2, sa.c1, sa.c2>;
        for (int x = 0; x < sa.c1; ++x)
            for (int z = 0; z < sa.c2; ++z) {
                T2 acc{0, 0};
                for (int i = 0; i < sa.s1; ++i) {
                    acc.x += a[I::at(i, i, x, z)].x;
                    acc.y += a[I::at(i, i, x, z)].y;
                }
                r[x * sa.c2 + z] = acc;
            }
    } else if constexpr (OP == K_REAL) {
        r[0] = T2{a[0].x, 0};
    } else if constexpr (OP == K_IMAG) {
        r[0] = T2{a[0].y, 0};
    } else if constexpr (OP == K_NORM2) {
        R acc = 0;
        for (int k = 0; k < NA; ++k) acc = fmadd(a[k].x, a[k].x, fmadd(a[k].y, a[k].y, acc));
        r[0] = T2{acc, 0};
    } else if constexpr (OP == K_INNER) {
        T2 acc{0, 0};
        for (int k = 0; k < NA; ++k) cmac_conj(acc, a[k], b[k]);
        r[0] = acc;
    } else if constexpr (OP == K_TRACE_MUL) {
        // Tr(a b) = sum a[i][k][x][z] b[k][i][z][x] (a, b square, one type)
        using I = Idx<sa.s1, sa.s2, sa.c1, sa.c2>;
        T2 acc{0, 0};
        for (int i = 0; i < sa.s1; ++i)
            for (int k = 0; k < sa.s2; ++k)
                for (int x = 0; x < sa.c1; ++x)
                    for (int z = 0; z < sa.c2; ++z) cmac(acc, a[I::at(i, k, x, z)], b[I::at(k, i, z, x)]);
        r[0] = acc;
    } else if constexpr (OP == K_GAMMA_L) {
        using I = Idx<sa.s1, sa.s2, sa.c1, sa.c2>;
        const int n = A.gamma_n;
        for (int i = 0; i < 4; ++i) {
            const int j = A.gt.perm[n][i];
            const int code = A.gt.code[n][i];
            for (int k = 0; k < sa.s2; ++k)
                for (int x = 0; x < sa.c1; ++x)
                    for (int z = 0; z < sa.c2; ++z) r[I::at(i, k, x, z)] = phase(code, a[I::at(j, k, x, z)]);
        }
    } else if constexpr (OP == K_GAMMA_R) {
        using I = Idx<sa.s1, sa.s2, sa.c1, sa.c2>;
        const int n = A.gamma_n;
        // (a Gamma)[i][k] = a[i][k'] Gamma[k'][k], k' = perm(k) (involution)
        for (int k = 0; k < 4; ++k) {
            const int kp = A.gt.perm[n][k];
            const int code = A.gt.code[n][kp];
            for (int i = 0; i < sa.s1; ++i)
                for (int x = 0; x < sa.c1; ++x)
                    for (int z = 0; z < sa.c2; ++z) r[I::at(i, k, x, z)] = phase(code, a[I::at(i, kp, x, z)]);
        }
    } else if constexpr (OP == K_ADD || OP == K_SUB) {
        for (int k = 0; k < NA; ++k) {
            if constexpr (OP == K_ADD) r[k] = T2{a[k].x + b[k].x, a[k].y + b[k].y};
            else r[k] = T2{a[k].x - b[k].x, a[k].y - b[k].y};
        }
    } else if constexpr (OP == K_MUL) {
        constexpr Pair ps = mul_part(sa.s1, sa.s2, sb.s1, sb.s2);
        constexpr Pair pc = mul_part(sa.c1, sa.c2, sb.c1, sb.c2);
        using IA = Idx<sa.s1, sa.s2, sa.c1, sa.c2>;
        using IB = Idx<sb.s1, sb.s2, sb.c1, sb.c2>;
        using IR = Idx<ps.r, ps.c, pc.r, pc.c>;
        constexpr bool aS = sa.s1 == 1 && sa.s2 == 1, bS = sb.s1 == 1 && sb.s2 == 1;
        constexpr bool aC = sa.c1 == 1 && sa.c2 == 1, bC = sb.c1 == 1 && sb.c2 == 1;
        constexpr int JS = (aS || bS) ? 1 : sa.s2;  // spin contraction length
        constexpr int JC = (aC || bC) ? 1 : sa.c2;  // colour contraction length
        for (int i = 0; i < ps.r; ++i)
            for (int k = 0; k < ps.c; ++k)
                for (int x = 0; x < pc.r; ++x)
                    for (int z = 0; z < pc.c; ++z) {
                        T2 acc{0, 0};
                        for (int j = 0; j < JS; ++j)
                            for (int y = 0; y < JC; ++y) {
                                const int ai = aS ? 0 : (bS ? i : i), ak = aS ? 0 : (bS ? k : j);
                                const int bi = bS ? 0 : (aS ? i : j), bk = bS ? 0 : k;
                                const int ax = aC ? 0 : x, az = aC ? 0 : (bC ? z : y);
                                const int bx = bC ? 0 : (aC ? x : y), bz = bC ? 0 : z;
                                cmac(acc, a[IA::at(ai, ak, ax, az)], b[IB::at(bi, bk, bx, bz)]);
                            }
                        r[IR::at(i, k, x, z)] = acc;
                    }
    }
}

template <int OP, int TA, int TB, typename R>
__global__ __launch_bounds__(256) void node_kernel(NodeArgs A) {
    using T2 = cplx_t<R>;
    constexpr int TR = result_type(OP, TA, TB);
    constexpr int NA = ncomp_of(TA), NB = is_binary(OP) ? ncomp_of(TB) : 1, NR = ncomp_of(TR);
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= A.sub.count) return;
    const int32_t s = (int32_t)subset_site(A.g, A.sub, l);
    int32_t c[4] = {0, 0, 0, 0};
    if (A.need_coords) cb_coords(A.g, s, c);
    T2 a[NA], b[NB], r[NR];
    load_operand<TA, R>(A.a, A.g, s, c, a);
    if constexpr (is_binary(OP)) load_operand<TB, R>(A.b, A.g, s, c, b);
    apply_op<OP, TA, TB, R>(A, a, b, r);
    store_values<R>(A.out, A.g, s, r, NR);
}

// Kernel table: [op][type a][type b][compute precision: 0 FP64, 1 FP32]
struct KernelTable {
    void* k[K_NUM_OPS][kNumTypes][kNumTypes][2];
};

template <int OP, int TA, int TB>
void fill_entry(KernelTable& t) {
    if constexpr (result_type(OP, TA, TB) >= 0 && (is_binary(OP) || TB == 0)) {
        t.k[OP][TA][TB][0] = reinterpret_cast<void*>(&node_kernel<OP, TA, TB, double>);
        t.k[OP][TA][TB][1] = reinterpret_cast<void*>(&node_kernel<OP, TA, TB, float>);
    }
}

template <int OP, int TA, int... TB>
void fill_tb(KernelTable& t, std::integer_sequence<int, TB...>) {
    (fill_entry<OP, TA, TB>(t), ...);
}

template <int OP, int... TA>
void fill_ta(KernelTable& t, std::integer_sequence<int, TA...>) {
    (fill_tb<OP, TA>(t, std::make_integer_sequence<int, kNumTypes>{}), ...);
}

template <int... OP>
void fill_ops(KernelTable& t, std::integer_sequence<int, OP...>) {
    (fill_ta<OP>(t, std::make_integer_sequence<int, kNumTypes>{}), ...);
}

const KernelTable& kernel_table() {
    static KernelTable table = [] {
        KernelTable t;
        std::memset(&t, 0, sizeof t);
        fill_ops(t, std::make_integer_sequence<int, K_NUM_OPS>{});
        return t;
    }();
    return table;
}

// Local-reduction kernels: [op][operand type] for the ops formed inside a
// reduction.
struct LocalReduceTable {
    void* k[K_NUM_OPS][kNumTypes];
};

template <int OP, int TA>
void fill_local(LocalReduceTable& t);

template <int OP, int... TA>
void fill_local_ta(LocalReduceTable& t, std::integer_sequence<int, TA...>) {
    (fill_local<OP, TA>(t), ...);
}

const LocalReduceTable& local_reduce_table();

// ---------------------------------------------------------------------------
// Fused stencil kernel: dest(x) = sum_k c_k [adj] M_k(x + d_k) V_k(x + e_k)
// ---------------------------------------------------------------------------

constexpr int kMaxTerms = 8;

struct StencilTerm {
    Operand mat;  // colour matrix (kind OPND_CONST: no matrix)
    Operand vec;
    int32_t has_mat, adj;
    double cre, cim;
};

struct StencilArgs {
    Geometry g;
    SubsetDesc sub;
    OutDesc out;
    int32_t nterms, need_coords;
    StencilTerm t[kMaxTerms];
};

template <typename R, int NSPIN>
__global__ __launch_bounds__(256) void stencil_kernel(StencilArgs A) {
    using T2 = cplx_t<R>;
    constexpr int NV = 3 * NSPIN;
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= A.sub.count) return;
    const int32_t s = (int32_t)subset_site(A.g, A.sub, l);
    int32_t c[4] = {0, 0, 0, 0};
    if (A.need_coords) cb_coords(A.g, s, c);
    T2 acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = T2{0, 0};
    for (int term = 0; term < A.nterms; ++term) {
        const StencilTerm& T = A.t[term];
        T2 v[NV];
        const int32_t vs = T.vec.has_disp ? displaced_site(A.g, c, T.vec.d) : s;
        load_comps<R, NV>(T.vec.base, T.vec.prec, T.vec.nrec, T.vec.ncomp, T.vec.rec, vs, v);
        T2 w[NV];
        if (T.has_mat) {
            T2 m[9];
            const int32_t ms = T.mat.has_disp ? displaced_site(A.g, c, T.mat.d) : s;
            load_comps<R, 9>(T.mat.base, T.mat.prec, T.mat.nrec, T.mat.ncomp, T.mat.rec, ms, m);
#pragma unroll
            for (int sp = 0; sp < NSPIN; ++sp)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    T2 t{0, 0};
                    if (T.adj) {
#pragma unroll
                        for (int b = 0; b < 3; ++b) cmac_conj(t, m[3 * b + a], v[3 * sp + b]);
                    } else {
#pragma unroll
                        for (int b = 0; b < 3; ++b) cmac(t, m[3 * a + b], v[3 * sp + b]);
                    }
                    w[3 * sp + a] = t;
                }
        } else {
#pragma unroll
            for (int k = 0; k < NV; ++k) w[k] = v[k];
        }
        const T2 coef{(R)T.cre, (R)T.cim};
#pragma unroll
        for (int k = 0; k < NV; ++k) cmac(acc[k], coef, w[k]);
    }
    store_values<R>(A.out, A.g, s, acc, NV);
}

// ---------------------------------------------------------------------------
// Reductions for qdp_sum_multi: per-component sums over the subsets of a set
// ---------------------------------------------------------------------------

struct ReduceArgs {
    Geometry g;
    const char* base;
    int32_t prec, nrec, ncomp, set;
    int32_t nchunks, pad;
    double* partial;  // [nsub][nchunks][ncomp][2]
};

__device__ __forceinline__ void set_subset(const Geometry& g, int32_t set, int32_t sub, SubsetDesc* d) {
    if (set == QDP_SET_ALL) *d = SubsetDesc{QDP_ALL, 0, g.V};
    else if (set == QDP_SET_PARITY) *d = SubsetDesc{sub == 0 ? QDP_EVEN : QDP_ODD, 0, g.Vh};
    else *d = SubsetDesc{QDP_TIMESLICE, sub, 2 * g.Vsh};
}

// Sum of NV complex values over the block's threads (wave shuffles, then
// the four waves in a fixed order); thread v < NV of wave 0 ends with value v.
template <int NV>
__device__ __forceinline__ void block_sum_values(double2 v[NV], double* lds /* [4][NV][2] */, double2* out) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            v[j].x += __shfl_xor(v[j].x, off, 64);
            v[j].y += __shfl_xor(v[j].y, off, 64);
        }
        if (lane == 0) {
            lds[(w * NV + j) * 2] = v[j].x;
            lds[(w * NV + j) * 2 + 1] = v[j].y;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < NV) {
        const int j = threadIdx.x;
        double re = 0.0, im = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            re += lds[(i * NV + j) * 2];
            im += lds[(i * NV + j) * 2 + 1];
        }
        *out = make_double2(re, im);
    }
}

// Per-component sums of a field, one thread per site and NV components
// (group blockIdx.z of the record: components z NV .. z NV + NV - 1), so a
// site's record is read once; FP64.
template <int NV>
__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs A) {
    const int chunk = blockIdx.x, sub = blockIdx.y, k0 = blockIdx.z * NV;
    SubsetDesc d;
    set_subset(A.g, A.set, sub, &d);
    double2 acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = make_double2(0.0, 0.0);
    for (int64_t l = (int64_t)chunk * blockDim.x + threadIdx.x; l < d.count; l += (int64_t)A.nchunks * blockDim.x) {
        const int32_t s = (int32_t)subset_site(A.g, d, l);
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            if (k0 + j < A.ncomp) {
                const double2 v = load_comp<double>(A.base, A.prec, A.nrec, A.ncomp, 0, k0 + j, s);
                acc[j].x += v.x;
                acc[j].y += v.y;
            }
        }
    }
    __shared__ double lds[4 * NV * 2];
    double2 r;
    block_sum_values<NV>(acc, lds, &r);
    if ((int)threadIdx.x < NV && k0 + (int)threadIdx.x < A.ncomp) {
        double* p = A.partial + (((int64_t)sub * A.nchunks + chunk) * A.ncomp + k0 + threadIdx.x) * 2;
        p[0] = r.x;
        p[1] = r.y;
    }
}

// Sums of a site-local scalar formed inside the reduction: OP = K_NORM2
// (sum |a|^2), K_INNER (sum a^dagger b), K_TRACE (trace a) or K_TRACE_MUL
// (trace a b) of operands of type TA, each read once at the sites of the set;
// no intermediate field.  FP64.
struct LocalReduceArgs {
    Geometry g;
    Operand a, b;
    int32_t set, nchunks;
    int32_t need_coords, pad;
    double* partial;  // [nsub][nchunks][1][2]
};

template <int OP, int TA>
__global__ __launch_bounds__(256) void reduce_local_kernel(LocalReduceArgs A) {
    constexpr int TB = is_binary(OP) ? TA : 0;
    constexpr int NA = ncomp_of(TA), NB = is_binary(OP) ? ncomp_of(TB) : 1;
    const int chunk = blockIdx.x, sub = blockIdx.y;
    SubsetDesc d;
    set_subset(A.g, A.set, sub, &d);
    const NodeArgs none{};
    double2 acc[1] = {make_double2(0.0, 0.0)};
    for (int64_t l = (int64_t)chunk * blockDim.x + threadIdx.x; l < d.count; l += (int64_t)A.nchunks * blockDim.x) {
        const int32_t s = (int32_t)subset_site(A.g, d, l);
        int32_t c[4] = {0, 0, 0, 0};
        if (A.need_coords) cb_coords(A.g, s, c);
        double2 a[NA], b[NB], r[1];
        load_operand<TA, double>(A.a, A.g, s, c, a);
        if constexpr (is_binary(OP)) load_operand<TB, double>(A.b, A.g, s, c, b);
        apply_op<OP, TA, TB, double>(none, a, b, r);
        acc[0].x += r[0].x;
        acc[0].y += r[0].y;
    }
    __shared__ double lds[8];
    double2 r;
    block_sum_values<1>(acc, lds, &r);
    if (threadIdx.x == 0) {
        double* p = A.partial + ((int64_t)sub * A.nchunks + chunk) * 2;
        p[0] = r.x;
        p[1] = r.y;
    }
}

// out[idx] for output idx = (subset, component): the sum of its partials over
// the chunks, one block of 256 threads per output.  Thread t adds chunks t,
// t + 256, ... in turn, then the 256 thread sums meet by a fixed tree (wave
// butterflies, then the four waves in order): the same order on every run.
// (A thread per output, walking up to 4097 chunks one after another, took
// about 0.3 ms, most of a global sum.)
__global__ __launch_bounds__(256) void reduce_finish(const double* __restrict__ partial, int32_t nsub,
                                                     int32_t nchunks, int32_t ncomp, double* __restrict__ out) {
    const int idx = blockIdx.x;
    const int sub = idx / ncomp, k = idx % ncomp;
    double re = 0.0, im = 0.0;
    for (int c = threadIdx.x; c < nchunks; c += 256) {
        const double* p = partial + (((int64_t)sub * nchunks + c) * ncomp + k) * 2;
        re += p[0];
        im += p[1];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_xor(re, off, 64);
        im += __shfl_xor(im, off, 64);
    }
    __shared__ double red[4][2];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w][0] = re;
        red[w][1] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[idx * 2] = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
        out[idx * 2 + 1] = (red[0][1] + red[1][1]) + (red[2][1] + red[3][1]);
    }
}

template <int OP, int TA>
void fill_local(LocalReduceTable& t) {
    constexpr int TB = is_binary(OP) ? TA : 0;
    if constexpr (result_type(OP, TA, TB) == QDP_REAL || result_type(OP, TA, TB) == QDP_COMPLEX)
        t.k[OP][TA] = reinterpret_cast<void*>(&reduce_local_kernel<OP, TA>);
}

const LocalReduceTable& local_reduce_table() {
    static LocalReduceTable table = [] {
        LocalReduceTable t;
        std::memset(&t, 0, sizeof t);
        fill_local_ta<K_NORM2>(t, std::make_integer_sequence<int, kNumTypes>{});
        fill_local_ta<K_INNER>(t, std::make_integer_sequence<int, kNumTypes>{});
        fill_local_ta<K_TRACE>(t, std::make_integer_sequence<int, kNumTypes>{});
        fill_local_ta<K_TRACE_MUL>(t, std::make_integer_sequence<int, kNumTypes>{});
        return t;
    }();
    return table;
}

// ---------------------------------------------------------------------------
// Host: parse, type-check, push shifts down, lower
// ---------------------------------------------------------------------------

namespace {

struct Node {
    int32_t op = -1;      // K_* for internal nodes, -1 leaf field, -2 constant
    int32_t type = -1;    // lattice type of the value
    uint64_t field = 0;   // leaf
    int32_t rec = 0;      // leaf: record (gauge direction)
    int32_t d[4] = {0, 0, 0, 0};
    double cre = 0, cim = 0;
    int32_t gamma_n = 0;
    std::unique_ptr<Node> a, b;
};

bool is_leaf(const Node& n) { return n.op < 0; }

qdp_status parse(Ctx* ctx, const qdp_expr* e, uint64_t lattice_hint, uint64_t* lattice,
                 std::unique_ptr<Node>* root) {
    std::vector<std::unique_ptr<Node>> st;
    uint64_t lat = lattice_hint;
    for (int32_t i = 0; i < e->n; ++i) {
        const qdp_node& q = e->nodes[i];
        auto n = std::make_unique<Node>();
        auto pop = [&](std::unique_ptr<Node>& dst) -> bool {
            if (st.empty()) return false;
            dst = std::move(st.back());
            st.pop_back();
            return true;
        };
        switch (q.op) {
            case QDP_OP_FIELD:
            case QDP_OP_GAUGE: {
                Field* f = find_field(ctx, q.field);
                if (!f) return set_error(ctx, QDP_ERR_STATE, "expr node %d: unknown field", i);
                if (lat && f->lattice != lat)
                    return set_error(ctx, QDP_ERR_LATTICE, "expr node %d: field on another lattice", i);
                lat = f->lattice;
                if (q.op == QDP_OP_GAUGE) {
                    if (f->type != QDP_GAUGE) return set_error(ctx, QDP_ERR_TYPE, "expr node %d: not a GAUGE field", i);
                    if (q.i0 < 0 || q.i0 > 3) return set_error(ctx, QDP_ERR_ARG, "expr node %d: mu out of range", i);
                    n->type = QDP_COLOR_MATRIX;
                    n->rec = q.i0;
                } else {
                    if (f->type == QDP_GAUGE)
                        return set_error(ctx, QDP_ERR_TYPE, "expr node %d: use QDP_OP_GAUGE for a gauge field", i);
                    n->type = f->type;
                }
                n->field = q.field;
                n->op = -1;
                break;
            }
            case QDP_OP_REAL_CONST:
            case QDP_OP_COMPLEX_CONST:
                n->op = -2;
                n->type = q.op == QDP_OP_REAL_CONST ? QDP_REAL : QDP_COMPLEX;
                n->cre = q.re;
                n->cim = q.op == QDP_OP_REAL_CONST ? 0.0 : q.im;
                break;
            case QDP_OP_SHIFT: {
                if (q.i0 < 0 || q.i0 > 3 || (q.i1 != 1 && q.i1 != -1))
                    return set_error(ctx, QDP_ERR_ARG, "expr node %d: shift needs mu 0..3, sign +1/-1", i);
                std::unique_ptr<Node> c;
                if (!pop(c)) return set_error(ctx, QDP_ERR_TYPE, "expr node %d: missing operand", i);
                // marker node, removed by the push-down pass
                n->op = 1000;
                n->type = c->type;
                n->d[q.i0] = q.i1;
                n->a = std::move(c);
                break;
            }
            default: {
                static const int map[] = {-1, -1, -1, -1, -1, K_NEG, K_CONJ, K_ADJ, K_ADD, K_SUB, K_MUL, K_GAMMA_L,
                                          K_GAMMA_R, K_TRACE, K_TRACE_COLOR, K_TRACE_SPIN, K_REAL, K_IMAG,
                                          K_NORM2, K_INNER};
                if (q.op < 0 || q.op > QDP_OP_LOCAL_INNER || map[q.op] < 0)
                    return set_error(ctx, QDP_ERR_ARG, "expr node %d: unknown op %d", i, q.op);
                n->op = map[q.op];
                if (is_binary(n->op)) {
                    if (!pop(n->b) || !pop(n->a)) return set_error(ctx, QDP_ERR_TYPE, "expr node %d: missing operand", i);
                } else if (!pop(n->a)) {
                    return set_error(ctx, QDP_ERR_TYPE, "expr node %d: missing operand", i);
                }
                if (n->op == K_GAMMA_L || n->op == K_GAMMA_R) {
                    if (q.i0 < 0 || q.i0 > 15) return set_error(ctx, QDP_ERR_ARG, "expr node %d: gamma index 0..15", i);
                    n->gamma_n = q.i0;
                }
                const int tb = n->b ? n->b->type : 0;
                n->type = result_type(n->op, n->a->type, tb);
                if (n->type < 0)
                    return set_error(ctx, QDP_ERR_TYPE, "expr node %d: op %d not defined for types %d, %d", i, q.op,
                                     n->a->type, tb);
            }
        }
        st.push_back(std::move(n));
    }
    if (st.size() != 1) return set_error(ctx, QDP_ERR_TYPE, "malformed expression (%zu values left)", st.size());
    *root = std::move(st.back());
    *lattice = lat;
    return QDP_OK;
}

// Remove shift markers, adding their displacement to every leaf below.
void push_down(std::unique_ptr<Node>& n, const int32_t d[4]) {
    if (n->op == 1000) {
        int32_t dd[4];
        for (int i = 0; i < 4; ++i) dd[i] = d[i] + n->d[i];
        std::unique_ptr<Node> child = std::move(n->a);
        push_down(child, dd);
        n = std::move(child);
        return;
    }
    if (is_leaf(*n)) {
        if (n->op == -1)
            for (int i = 0; i < 4; ++i) n->d[i] += d[i];
        return;
    }
    if (n->a) push_down(n->a, d);
    if (n->b) push_down(n->b, d);
}

bool has_disp(const Node& n) { return n.d[0] || n.d[1] || n.d[2] || n.d[3]; }

bool reads_shifted(const Node& n, uint64_t id) {
    if (n.op == -1) return n.field == id && has_disp(n);
    return (n.a && reads_shifted(*n.a, id)) || (n.b && reads_shifted(*n.b, id));
}

bool any_disp(const Node& n) {
    if (n.op == -1) return has_disp(n);
    return (n.a && any_disp(*n.a)) || (n.b && any_disp(*n.b));
}

// Reduce a displacement modulo the extents (shifts may wrap several times).
void normalise(const Geometry& g, int32_t d[4]) {
    for (int mu = 0; mu < 4; ++mu) {
        d[mu] %= g.L[mu];
        if (d[mu] < 0) d[mu] += g.L[mu];
    }
}

// --- fused stencil matching -------------------------------------------------

struct Term {
    const Node* mat = nullptr;
    bool adj = false;
    const Node* vec = nullptr;
    double cre = 1, cim = 0;
};

bool collect_terms(const Node& n, double cre, double cim, int vec_type, std::vector<Term>& out);

// term := const * term | term * const | [adj](M) * V | V | -term
bool match_product(const Node& n, double cre, double cim, int vec_type, Term& t) {
    if (n.op == K_NEG) return match_product(*n.a, -cre, -cim, vec_type, t);
    if (n.op == -1 && n.type == vec_type) {
        t.vec = &n;
        t.cre = cre;
        t.cim = cim;
        return true;
    }
    if (n.op != K_MUL) return false;
    const Node& A = *n.a;
    const Node& B = *n.b;
    if (A.op == -2) {
        const double r = cre * A.cre - cim * A.cim, i = cre * A.cim + cim * A.cre;
        return match_product(B, r, i, vec_type, t);
    }
    if (B.op == -2) {
        const double r = cre * B.cre - cim * B.cim, i = cre * B.cim + cim * B.cre;
        return match_product(A, r, i, vec_type, t);
    }
    const Node* m = &A;
    bool adj = false;
    if (m->op == K_ADJ) {
        adj = true;
        m = m->a.get();
    }
    if (m->op != -1 || m->type != QDP_COLOR_MATRIX || B.op != -1 || B.type != vec_type) return false;
    t.mat = m;
    t.adj = adj;
    t.vec = &B;
    t.cre = cre;
    t.cim = cim;
    return true;
}

bool collect_terms(const Node& n, double cre, double cim, int vec_type, std::vector<Term>& out) {
    if (n.op == K_ADD || n.op == K_SUB) {
        if (!collect_terms(*n.a, cre, cim, vec_type, out)) return false;
        return collect_terms(*n.b, n.op == K_SUB ? -cre : cre, n.op == K_SUB ? -cim : cim, vec_type, out);
    }
    if (n.op == K_MUL && (n.a->op == -2 || n.b->op == -2)) {
        const Node& c = n.a->op == -2 ? *n.a : *n.b;
        const Node& x = n.a->op == -2 ? *n.b : *n.a;
        if (x.op == K_ADD || x.op == K_SUB || x.op == K_MUL || x.op == K_NEG) {
            const double r = cre * c.cre - cim * c.cim, i = cre * c.cim + cim * c.cre;
            return collect_terms(x, r, i, vec_type, out);
        }
    }
    if (n.op == K_NEG) return collect_terms(*n.a, -cre, -cim, vec_type, out);
    Term t;
    if (!match_product(n, cre, cim, vec_type, t)) return false;
    out.push_back(t);
    return out.size() <= (size_t)kMaxTerms;
}

// --- operand descriptors ---------------------------------------------------

struct Lowering {
    Ctx* ctx;
    const Geometry* g;
    PinSet* pins;
    std::vector<std::unique_ptr<PoolTemp>> temps;
    GammaTab gt;
};

qdp_status leaf_operand(Lowering& L, const Node& n, Operand* op) {
    std::memset(op, 0, sizeof *op);
    if (n.op == -2) {
        op->kind = OPND_CONST;
        op->cre = n.cre;
        op->cim = n.cim;
        return QDP_OK;
    }
    Field* f = find_field(L.ctx, n.field);
    char* p;
    QDP_CHECK(L.pins->add(n.field, true, &p));
    const TypeShape ts = type_shape(f->type);
    op->base = p;
    op->kind = OPND_FIELD;
    op->prec = f->prec;
    op->rec = n.rec;
    op->nrec = ts.nrec;
    op->ncomp = ts.ncomp;
    int32_t d[4] = {n.d[0], n.d[1], n.d[2], n.d[3]};
    normalise(*L.g, d);
    for (int i = 0; i < 4; ++i) op->d[i] = d[i];
    op->has_disp = d[0] || d[1] || d[2] || d[3];
    return QDP_OK;
}

qdp_status temp_operand(Lowering& L, int type, int prec, Operand* op, OutDesc* out) {
    auto t = std::make_unique<PoolTemp>();
    QDP_CHECK(t->alloc(L.ctx, field_bytes(*L.g, type, prec)));
    const TypeShape ts = type_shape(type);
    std::memset(op, 0, sizeof *op);
    op->base = t->ptr();
    op->kind = OPND_FIELD;
    op->prec = prec;
    op->nrec = ts.nrec;
    op->ncomp = ts.ncomp;
    out->base = t->ptr();
    out->prec = prec;
    out->nrec = ts.nrec;
    out->ncomp = ts.ncomp;
    out->real_only = type == QDP_REAL;
    L.temps.push_back(std::move(t));
    return QDP_OK;
}

// Evaluate node n into `out` (a temporary or the destination).
// trace(a b) of two square matrices of one type (colour, spin or
// propagator): evaluated as one node, Tr(a b) = sum a_ij b_ji.
bool is_trace_of_product(const Node& n) {
    if (n.op != K_TRACE || !n.a || n.a->op != K_MUL) return false;
    const Node& m = *n.a;
    return result_type(K_TRACE_MUL, m.a->type, m.b->type) >= 0;
}

qdp_status emit(Lowering& L, const Node& n, const SubsetDesc& sub, const OutDesc& out, int cprec) {
    NodeArgs A;
    std::memset(&A, 0, sizeof A);
    A.g = *L.g;
    A.sub = sub;
    A.out = out;
    A.gt = L.gt;
    int op = n.op, ta = n.type, tb = 0;
    const Node* na = &n;
    const Node* nb = nullptr;
    if (is_leaf(n)) {
        op = K_COPY;
    } else if (is_trace_of_product(n)) {
        // trace(a b) in one kernel: no product field in between
        op = K_TRACE_MUL;
        na = n.a->a.get();
        nb = n.a->b.get();
        ta = tb = na->type;
    } else {
        na = n.a.get();
        nb = n.b.get();
        ta = na->type;
        tb = nb ? nb->type : 0;
        A.gamma_n = n.gamma_n;
    }
    auto operand = [&](const Node& c, Operand* o) -> qdp_status {
        if (is_leaf(c)) return leaf_operand(L, c, o);
        OutDesc tmp;
        QDP_CHECK(temp_operand(L, c.type, cprec, o, &tmp));
        return emit(L, c, sub, tmp, cprec);
    };
    QDP_CHECK(operand(*na, &A.a));
    if (nb) QDP_CHECK(operand(*nb, &A.b));
    A.need_coords = A.a.has_disp || (nb && A.b.has_disp);
    void* fn = kernel_table().k[op][ta][tb][cprec == QDP_F64 ? 0 : 1];
    if (!fn) return set_error(L.ctx, QDP_ERR_TYPE, "no kernel for op %d on types %d, %d", op, ta, tb);
    if (sub.count == 0) return QDP_OK;
    void* args[] = {&A};
    QDP_HIP(L.ctx, hipLaunchKernel(fn, dim3((unsigned)((sub.count + 255) / 256)), dim3(256), args, 0, L.ctx->stream));
    return check_launch(L.ctx, "expression node kernel");
}

qdp_status emit_stencil(Lowering& L, const std::vector<Term>& terms, int vec_type, const SubsetDesc& sub,
                        const OutDesc& out, int cprec) {
    StencilArgs A;
    std::memset(&A, 0, sizeof A);
    A.g = *L.g;
    A.sub = sub;
    A.out = out;
    A.nterms = (int32_t)terms.size();
    for (size_t k = 0; k < terms.size(); ++k) {
        StencilTerm& T = A.t[k];
        QDP_CHECK(leaf_operand(L, *terms[k].vec, &T.vec));
        if (terms[k].mat) {
            QDP_CHECK(leaf_operand(L, *terms[k].mat, &T.mat));
            T.has_mat = 1;
            T.adj = terms[k].adj;
        }
        T.cre = terms[k].cre;
        T.cim = terms[k].cim;
        if (T.vec.has_disp || (T.has_mat && T.mat.has_disp)) A.need_coords = 1;
    }
    if (sub.count == 0) return QDP_OK;
    void* fn;
    if (vec_type == QDP_FERMION)
        fn = cprec == QDP_F64 ? reinterpret_cast<void*>(&stencil_kernel<double, 4>)
                              : reinterpret_cast<void*>(&stencil_kernel<float, 4>);
    else
        fn = cprec == QDP_F64 ? reinterpret_cast<void*>(&stencil_kernel<double, 1>)
                              : reinterpret_cast<void*>(&stencil_kernel<float, 1>);
    void* args[] = {&A};
    QDP_HIP(L.ctx, hipLaunchKernel(fn, dim3((unsigned)((sub.count + 255) / 256)), dim3(256), args, 0, L.ctx->stream));
    return check_launch(L.ctx, "stencil kernel");
}

GammaTab gamma_tab(Ctx* ctx) {
    // Signed permutation of every Gamma_n from the context's tables.
    GammaTab t;
    for (int sg = 0; sg < 4; ++sg)
        for (int m = 0; m < 4; ++m) {
            const int n = ctx->gamma.group_members[sg][m];
            for (int r = 0; r < 4; ++r) {
                t.perm[n][r] = (int8_t)ctx->gamma.group_perm[sg][r];
                // P_n[r] = s_r Gamma_n[r, sigma r]; undo s_r to get Gamma_n's code
                const double* ph = ctx->gamma.p_phase[n][r];
                int code = ph[0] > 0.5 ? 0 : ph[1] > 0.5 ? 1 : ph[0] < -0.5 ? 2 : 3;
                if (r >= 2) code = (code + 2) & 3;
                t.code[n][r] = (int8_t)code;
            }
        }
    return t;
}

SubsetDesc subset_desc(const Geometry& g, qdp_subset s) {
    switch (s.kind) {
        case QDP_EVEN: return SubsetDesc{QDP_EVEN, 0, g.Vh};
        case QDP_ODD: return SubsetDesc{QDP_ODD, 0, g.Vh};
        case QDP_TIMESLICE: return SubsetDesc{QDP_TIMESLICE, s.t, 2 * g.Vsh};
        default: return SubsetDesc{QDP_ALL, 0, g.V};
    }
}

// Shared front end of eval and sum_multi.
qdp_status build_tree(Ctx* ctx, const qdp_expr* expr, uint64_t lattice_hint, uint64_t* lattice,
                      std::unique_ptr<Node>* root) {
    QDP_CHECK(parse(ctx, expr, lattice_hint, lattice, root));
    if (!*lattice) return set_error(ctx, QDP_ERR_TYPE, "expression reads no lattice field");
    const int32_t zero[4] = {0, 0, 0, 0};
    push_down(*root, zero);
    return QDP_OK;
}

}  // namespace

qdp_status eval_impl(Ctx* ctx, const qdp_expr* expr, uint64_t dest, qdp_subset subset, int32_t assign) {
    Field* df = find_field(ctx, dest);
    if (!df) return set_error(ctx, QDP_ERR_STATE, "eval: unknown destination");
    if (df->type == QDP_GAUGE) return set_error(ctx, QDP_ERR_TYPE, "eval: GAUGE destination");
    if (assign < QDP_ASSIGN || assign > QDP_MUL_ASSIGN) return set_error(ctx, QDP_ERR_ARG, "eval: bad assign op");
    if (subset.kind < QDP_ALL || subset.kind > QDP_TIMESLICE) return set_error(ctx, QDP_ERR_ARG, "eval: bad subset");
    uint64_t lat = 0;
    std::unique_ptr<Node> root;
    QDP_CHECK(build_tree(ctx, expr, df->lattice, &lat, &root));
    const Geometry g = find_lattice(ctx, lat)->geo;
    if (subset.kind == QDP_TIMESLICE && (subset.t < 0 || subset.t >= g.L[3]))
        return set_error(ctx, QDP_ERR_ARG, "eval: time slice out of range");
    if (assign != QDP_ASSIGN) {
        auto d = std::make_unique<Node>();
        d->op = -1;
        d->type = df->type;
        d->field = dest;
        auto top = std::make_unique<Node>();
        top->op = assign == QDP_ADD_ASSIGN ? K_ADD : assign == QDP_SUB_ASSIGN ? K_SUB : K_MUL;
        top->type = result_type(top->op, df->type, root->type);
        if (top->type < 0) return set_error(ctx, QDP_ERR_TYPE, "eval: compound assignment type mismatch");
        top->a = std::move(d);
        top->b = std::move(root);
        root = std::move(top);
    }
    if (!(root->type == df->type || (root->type == QDP_REAL && df->type == QDP_COMPLEX)))
        return set_error(ctx, QDP_ERR_TYPE, "eval: cannot assign type %d to a field of type %d", root->type, df->type);
    if (reads_shifted(*root, dest))
        return set_error(ctx, QDP_ERR_ALIAS, "eval: destination is read at a shifted site");

    PinSet pins(ctx);
    Lowering L{ctx, &g, &pins, {}, gamma_tab(ctx)};
    char* pd;
    QDP_CHECK(pins.add(dest, true, &pd));
    const TypeShape ts = type_shape(df->type);
    OutDesc out{pd, df->prec, ts.nrec, ts.ncomp, df->type == QDP_REAL};
    const SubsetDesc sub = subset_desc(g, subset);
    const int cprec = df->prec == QDP_F64 ? QDP_F64 : QDP_F32;

    if (df->type == QDP_FERMION || df->type == QDP_COLOR_VECTOR) {
        std::vector<Term> terms;
        if (collect_terms(*root, 1.0, 0.0, df->type, terms) && !terms.empty())
            return emit_stencil(L, terms, df->type, sub, out, cprec);
    }
    return emit(L, *root, sub, out, cprec);
}

qdp_status sum_multi_impl(Ctx* ctx, const qdp_expr* expr, int32_t set, double* out, size_t n_doubles) {
    if (set < QDP_SET_ALL || set > QDP_SET_TIMESLICE) return set_error(ctx, QDP_ERR_ARG, "sum_multi: bad set");
    uint64_t lat = 0;
    std::unique_ptr<Node> root;
    QDP_CHECK(build_tree(ctx, expr, 0, &lat, &root));
    const Geometry g = find_lattice(ctx, lat)->geo;
    const int type = root->type;
    const TypeShape ts = type_shape(type);
    const int nsub = set == QDP_SET_ALL ? 1 : set == QDP_SET_PARITY ? 2 : g.L[3];
    const size_t need = (size_t)nsub * ts.ncomp * 2;
    if (n_doubles < need) return set_error(ctx, QDP_ERR_ARG, "sum_multi: output needs %zu doubles", need);

    PinSet pins(ctx);
    Lowering L{ctx, &g, &pins, {}, gamma_tab(ctx)};
    ReduceArgs R;
    std::memset(&R, 0, sizeof R);
    R.g = g;
    R.ncomp = ts.ncomp;
    R.nrec = ts.nrec;
    R.set = set;
    int64_t per_sub = set == QDP_SET_ALL ? g.V : set == QDP_SET_PARITY ? g.Vh : 2 * g.Vsh;
    // enough blocks to keep every CU's memory pipeline busy (about 16 waves
    // per CU over all subsets), each thread then walking its chunk's sites
    int64_t nchunks = std::max<int64_t>(1, std::min<int64_t>((per_sub + 255) / 256, 4096 / nsub + 1));
    R.nchunks = (int32_t)nchunks;
    PoolTemp scratch;
    const size_t partial_bytes = sizeof(double) * 2 * (size_t)nsub * nchunks * ts.ncomp;
    QDP_CHECK(scratch.alloc(ctx, (int64_t)(partial_bytes + need * sizeof(double) + 256)));
    R.partial = reinterpret_cast<double*>(scratch.ptr());
    double* d_out = reinterpret_cast<double*>(scratch.ptr() + ((partial_bytes + 255) & ~size_t(255)));

    // a site-local scalar (|a|^2, a^dagger b, trace a, trace a b) is formed
    // inside the reduction, its operands evaluated first only if they are
    // not fields
    int lop = -1, lta = 0;
    const Node *la = nullptr, *lb = nullptr;
    if (is_trace_of_product(*root)) {
        lop = K_TRACE_MUL;
        la = root->a->a.get();
        lb = root->a->b.get();
    } else if (root->op == K_NORM2 || root->op == K_INNER || root->op == K_TRACE) {
        lop = root->op;
        la = root->a.get();
        lb = root->b.get();
    }
    if (la) lta = la->type;
    void* lfn = lop >= 0 ? local_reduce_table().k[lop][lta] : nullptr;
    if (lfn) {
        LocalReduceArgs LA;
        std::memset(&LA, 0, sizeof LA);
        LA.g = g;
        LA.set = set;
        LA.nchunks = (int32_t)nchunks;
        LA.partial = R.partial;
        auto operand = [&](const Node& c, Operand* o) -> qdp_status {
            if (is_leaf(c)) return leaf_operand(L, c, o);
            OutDesc tmp;
            QDP_CHECK(temp_operand(L, c.type, QDP_F64, o, &tmp));
            return emit(L, c, SubsetDesc{QDP_ALL, 0, g.V}, tmp, QDP_F64);
        };
        QDP_CHECK(operand(*la, &LA.a));
        if (lb) QDP_CHECK(operand(*lb, &LA.b));
        LA.need_coords = LA.a.has_disp || (lb && LA.b.has_disp);
        void* args[] = {&LA};
        QDP_HIP(ctx, hipLaunchKernel(lfn, dim3((unsigned)nchunks, nsub, 1), dim3(256), args, 0, ctx->stream));
        QDP_CHECK(check_launch(ctx, "local reduce kernel"));
    } else {
        if (root->op == -1 && !has_disp(*root) && find_field(ctx, root->field)->type == root->type) {
            // a bare field: reduce it in place
            Operand o;
            QDP_CHECK(leaf_operand(L, *root, &o));
            R.base = o.base;
            R.prec = o.prec;
        } else {
            // evaluate the expression in FP64 over all sites into a temporary
            Operand o;
            OutDesc tmp;
            QDP_CHECK(temp_operand(L, type, QDP_F64, &o, &tmp));
            QDP_CHECK(emit(L, *root, SubsetDesc{QDP_ALL, 0, g.V}, tmp, QDP_F64));
            R.base = o.base;
            R.prec = QDP_F64;
        }
        // one thread per site and up to 16 components (propagators: nine
        // groups, each reading its part of the record)
        const int nv = ts.ncomp <= 16 ? ts.ncomp : 16;
        const int ngroups = (ts.ncomp + nv - 1) / nv;
        void* fn = nv == 1 ? reinterpret_cast<void*>(&reduce_kernel<1>)
                 : nv == 3 ? reinterpret_cast<void*>(&reduce_kernel<3>)
                 : nv == 9 ? reinterpret_cast<void*>(&reduce_kernel<9>)
                 : nv == 12 ? reinterpret_cast<void*>(&reduce_kernel<12>)
                            : reinterpret_cast<void*>(&reduce_kernel<16>);
        void* args[] = {&R};
        QDP_HIP(ctx, hipLaunchKernel(fn, dim3((unsigned)nchunks, nsub, ngroups), dim3(256), args, 0, ctx->stream));
        QDP_CHECK(check_launch(ctx, "reduce kernel"));
    }
    const int nt = nsub * ts.ncomp;
    hipLaunchKernelGGL(reduce_finish, dim3(nt), dim3(256), 0, ctx->stream, R.partial, nsub, (int32_t)nchunks,
                       ts.ncomp, d_out);
    QDP_CHECK(check_launch(ctx, "reduce finish kernel"));
    double* host;
    QDP_CHECK(host_result_buffer(ctx, need * sizeof(double), &host));
    QDP_HIP(ctx, hipMemcpyAsync(host, d_out, need * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    QDP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::memcpy(out, host, need * sizeof(double));
    return QDP_OK;
}

}  // namespace qdpmi
