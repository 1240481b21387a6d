/*
 * FP64 CPU oracle for Jacobi smearing, meson contractions and lattice sums.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  It is built by the repository's build step
 * (gcc) and loaded only by the tests, the smoke check and the CPU-baseline leg
 * of the benchmark.  The GPU library never links, loads or calls it, and it
 * includes nothing from the GPU library.
 *
 * Everything is double precision and uses the canonical host layouts:
 *   site index      s = x + Lx*(y + Ly*(z + Lz*t)), periodic in every direction
 *   complex         interleaved (re, im) doubles
 *   colour matrix   [site][row 3][col 3]
 *   gauge field     [mu 4][site][row 3][col 3], mu = 0,1,2 spatial, mu = 3 time
 *   fermion column  [site][spin 4][colour 3]
 *   propagator      12 fermion columns, column j = 3*spin_src + colour_src
 *
 * Paper context (Winter, "Accelerating QDP++/Chroma on GPUs", Lattice 2011):
 * section 5 lists the measured chain as source creation, source smearing,
 * propagator, sink smearing and the mesonic hadron spectrum; section 4 states
 * that expressions are evaluated site by site over lattice objects.  The paper
 * does not print the smearing operator or the contraction formula; the
 * readings used here are listed in the header of each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double re, im;
} cplx;

static inline cplx c_make(double re, double im) { cplx c = {re, im}; return c; }
static inline cplx c_add(cplx a, cplx b) { return c_make(a.re + b.re, a.im + b.im); }
static inline cplx c_mul(cplx a, cplx b) {
    return c_make(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
static inline cplx c_conj(cplx a) { return c_make(a.re, -a.im); }
static inline cplx c_scale(double s, cplx a) { return c_make(s * a.re, s * a.im); }

/* ------------------------------------------------------------------------ */
/* Geometry: lexicographic sites, x fastest, periodic boundaries.            */
/* ------------------------------------------------------------------------ */

static int64_t volume(const int32_t d[4]) {
    return (int64_t)d[0] * d[1] * d[2] * d[3];
}

static void site_coords(const int32_t d[4], int64_t s, int32_t c[4]) {
    for (int mu = 0; mu < 4; ++mu) {
        c[mu] = (int32_t)(s % d[mu]);
        s /= d[mu];
    }
}

static int64_t site_index(const int32_t d[4], const int32_t c[4]) {
    int64_t s = 0;
    for (int mu = 3; mu >= 0; --mu) s = s * d[mu] + c[mu];
    return s;
}

/* Site reached from s by moving `step` lattice units along direction mu,
 * wrapping periodically. */
static int64_t neighbour(const int32_t d[4], int64_t s, int mu, int step) {
    int32_t c[4];
    site_coords(d, s, c);
    int32_t v = (c[mu] + step) % d[mu];
    if (v < 0) v += d[mu];
    c[mu] = v;
    return site_index(d, c);
}

int64_t or_neighbour(const int32_t d[4], int64_t s, int32_t mu, int32_t step) {
    return neighbour(d, s, mu, step);
}

/* ------------------------------------------------------------------------ */
/* Shift: dest(x) = src(x + sign * mu_hat), for a field of `ncomplex`        */
/* complex numbers per site.  This is the QDP shift() the paper's expression */
/* engine supports (section 4.2: expressions over lattice objects).          */
/* ------------------------------------------------------------------------ */

void or_shift(const int32_t d[4], int32_t ncomplex, const double* src, double* dst,
              int32_t mu, int32_t sign) {
    const int64_t V = volume(d);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        const int64_t from = neighbour(d, s, mu, sign);
        memcpy(dst + 2 * ncomplex * s, src + 2 * ncomplex * from,
               sizeof(double) * 2 * ncomplex);
    }
}

/* ------------------------------------------------------------------------ */
/* Jacobi smearing.                                                          */
/*                                                                           */
/* Reading (the paper names source and sink smearing, SRC and SNK in         */
/* section 5 and Figure 4, without writing the operator down): the smeared   */
/* field is (1 + kappa*H)^N psi with the gauge-covariant spatial hopping     */
/*   (H psi)(x) = sum_{i=0,1,2} [ U_i(x) psi(x+i) + U_i(x-i)^dagger psi(x-i) ]*/
/* acting on colour and as the identity on spin.  No normalisation between   */
/* steps.  Time slices never mix.  For a unit gauge field the plane wave of  */
/* spatial momentum p is an eigenvector with eigenvalue 1 + 2 kappa sum cos. */
/* ------------------------------------------------------------------------ */

/* w = U v  (colour matrix times colour vector) */
static void mat_vec(const double* U, const double* v, cplx w[3]) {
    for (int a = 0; a < 3; ++a) {
        cplx acc = c_make(0.0, 0.0);
        for (int b = 0; b < 3; ++b) {
            const cplx u = c_make(U[2 * (3 * a + b)], U[2 * (3 * a + b) + 1]);
            const cplx x = c_make(v[2 * b], v[2 * b + 1]);
            acc = c_add(acc, c_mul(u, x));
        }
        w[a] = acc;
    }
}

/* w = U^dagger v */
static void adj_mat_vec(const double* U, const double* v, cplx w[3]) {
    for (int a = 0; a < 3; ++a) {
        cplx acc = c_make(0.0, 0.0);
        for (int b = 0; b < 3; ++b) {
            const cplx u = c_make(U[2 * (3 * b + a)], U[2 * (3 * b + a) + 1]);
            const cplx x = c_make(v[2 * b], v[2 * b + 1]);
            acc = c_add(acc, c_mul(c_conj(u), x));
        }
        w[a] = acc;
    }
}

/* (H psi)(s) for one fermion column, 12 complex numbers written to h. */
static void hopping_at(const int32_t d[4], const double* U, const double* psi,
                       int64_t s, cplx h[12]) {
    const int64_t V = volume(d);
    for (int k = 0; k < 12; ++k) h[k] = c_make(0.0, 0.0);
    for (int i = 0; i < 3; ++i) {
        const int64_t fwd = neighbour(d, s, i, +1);
        const int64_t bwd = neighbour(d, s, i, -1);
        const double* U_here = U + 18 * ((int64_t)i * V + s);
        const double* U_back = U + 18 * ((int64_t)i * V + bwd);
        for (int spin = 0; spin < 4; ++spin) {
            cplx w[3];
            mat_vec(U_here, psi + 24 * fwd + 6 * spin, w);
            for (int a = 0; a < 3; ++a) h[3 * spin + a] = c_add(h[3 * spin + a], w[a]);
            adj_mat_vec(U_back, psi + 24 * bwd + 6 * spin, w);
            for (int a = 0; a < 3; ++a) h[3 * spin + a] = c_add(h[3 * spin + a], w[a]);
        }
    }
}

/* One application of (1 + kappa H) to one fermion column. */
void or_smear_step(const int32_t d[4], const double* U, const double* psi,
                   double* out, double kappa) {
    const int64_t V = volume(d);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        cplx h[12];
        hopping_at(d, U, psi, s, h);
        for (int k = 0; k < 12; ++k) {
            out[24 * s + 2 * k] = psi[24 * s + 2 * k] + kappa * h[k].re;
            out[24 * s + 2 * k + 1] = psi[24 * s + 2 * k + 1] + kappa * h[k].im;
        }
    }
}

/* psi_out = (1 + kappa H)^niter psi_in for `ncols` fermion columns stored one
 * after another ([col][site][spin][colour]).  psi_in and psi_out may alias. */
int32_t or_smear(const int32_t d[4], const double* U, const double* psi_in,
                 double* psi_out, double kappa, int32_t niter, int32_t ncols) {
    const int64_t V = volume(d);
    const size_t col_doubles = (size_t)24 * V;
    double* a = (double*)malloc(sizeof(double) * col_doubles);
    double* b = (double*)malloc(sizeof(double) * col_doubles);
    if (!a || !b) {
        free(a);
        free(b);
        return -1;
    }
    for (int32_t c = 0; c < ncols; ++c) {
        memcpy(a, psi_in + c * col_doubles, sizeof(double) * col_doubles);
        for (int32_t k = 0; k < niter; ++k) {
            or_smear_step(d, U, a, b, kappa);
            double* t = a;
            a = b;
            b = t;
        }
        memcpy(psi_out + c * col_doubles, a, sizeof(double) * col_doubles);
    }
    free(a);
    free(b);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Gamma matrices, DeGrand-Rossi basis, written out as dense 4x4 complex     */
/* matrices.  Gamma_n = g1^b0 g2^b1 g3^b2 g4^b3 with b_k the bits of n, so   */
/* Gamma_15 = g1 g2 g3 g4 = gamma_5 = diag(1, 1, -1, -1).                    */
/* ------------------------------------------------------------------------ */

static void gamma_basis(int k, cplx g[4][4]) {
    memset(g, 0, sizeof(cplx) * 16);
    const cplx I = c_make(0.0, 1.0), mI = c_make(0.0, -1.0);
    const cplx one = c_make(1.0, 0.0), mone = c_make(-1.0, 0.0);
    switch (k) {
        case 0: /* gamma_1 */
            g[0][3] = I; g[1][2] = I; g[2][1] = mI; g[3][0] = mI;
            break;
        case 1: /* gamma_2 */
            g[0][3] = mone; g[1][2] = one; g[2][1] = one; g[3][0] = mone;
            break;
        case 2: /* gamma_3 */
            g[0][2] = I; g[1][3] = mI; g[2][0] = mI; g[3][1] = I;
            break;
        default: /* gamma_4 */
            g[0][2] = one; g[1][3] = one; g[2][0] = one; g[3][1] = one;
            break;
    }
}

static void mat4_mul(cplx a[4][4], cplx b[4][4], cplx out[4][4]) {
    cplx r[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx acc = c_make(0.0, 0.0);
            for (int k = 0; k < 4; ++k) acc = c_add(acc, c_mul(a[i][k], b[k][j]));
            r[i][j] = acc;
        }
    memcpy(out, r, sizeof(r));
}

static void gamma_n(int n, cplx G[4][4]) {
    memset(G, 0, sizeof(cplx) * 16);
    for (int i = 0; i < 4; ++i) G[i][i] = c_make(1.0, 0.0);
    for (int k = 0; k < 4; ++k) {
        if (n & (1 << k)) {
            cplx g[4][4];
            gamma_basis(k, g);
            mat4_mul(G, g, G);
        }
    }
}

/* Dense Gamma_n as 16 interleaved complex numbers, row-major. */
void or_gamma(int32_t n, double* out) {
    cplx G[4][4];
    gamma_n(n, G);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            out[2 * (4 * i + j)] = G[i][j].re;
            out[2 * (4 * i + j) + 1] = G[i][j].im;
        }
}

/* ------------------------------------------------------------------------ */
/* Meson two-point functions (the mesonic hadron spectrum, HAD, of section 5)*/
/*                                                                           */
/*   C_n(t) = sum_{x : x_3 = t} Tr[ g5 S2(x)^dagger g5 Gamma_n S1(x) Gamma_n ]*/
/*                                                                           */
/* S(x) is the 12x12 matrix with rows = sink (spin, colour) and columns =    */
/* source j = 3*spin + colour, i.e. S[(alpha a),(beta b)] is component       */
/* (alpha, a) of column 3*beta + b.  No fermion-loop sign, zero momentum,    */
/* absolute time index.  out is [16][Lt][re, im].                            */
/* ------------------------------------------------------------------------ */

static inline cplx prop_elem(const double* S, int64_t V, int64_t s, int row, int col) {
    /* row = 3*alpha + a (sink), col = 3*beta + b (source) */
    const double* p = S + (size_t)col * 24 * V + 24 * s + 2 * row;
    return c_make(p[0], p[1]);
}

/* The 16 traces at every site: site_val[16 s + n]. */
static void meson_site_values(const int32_t d[4], const double* S1, const double* S2, cplx* site_val) {
    const int64_t V = volume(d);
    cplx G[16][4][4];
    for (int n = 0; n < 16; ++n) gamma_n(n, G[n]);
    const double g5[4] = {1.0, 1.0, -1.0, -1.0};

#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        cplx A[12][12]; /* g5 S2^dagger g5 */
        cplx B1[12][12];
        for (int r = 0; r < 12; ++r)
            for (int c = 0; c < 12; ++c) {
                /* (S2^dagger)[r][c] = conj(S2[c][r]) */
                const cplx v = c_conj(prop_elem(S2, V, s, c, r));
                A[r][c] = c_scale(g5[r / 3] * g5[c / 3], v);
                B1[r][c] = prop_elem(S1, V, s, r, c);
            }
        for (int n = 0; n < 16; ++n) {
            /* B = (Gamma_n x 1_colour) S1 (Gamma_n x 1_colour) */
            cplx T[12][12], B[12][12];
            for (int r = 0; r < 12; ++r)
                for (int c = 0; c < 12; ++c) {
                    cplx acc = c_make(0.0, 0.0);
                    for (int g = 0; g < 4; ++g)
                        acc = c_add(acc, c_mul(G[n][r / 3][g], B1[3 * g + r % 3][c]));
                    T[r][c] = acc;
                }
            for (int r = 0; r < 12; ++r)
                for (int c = 0; c < 12; ++c) {
                    cplx acc = c_make(0.0, 0.0);
                    for (int g = 0; g < 4; ++g)
                        acc = c_add(acc, c_mul(T[r][3 * g + c % 3], G[n][g][c / 3]));
                    B[r][c] = acc;
                }
            cplx tr = c_make(0.0, 0.0);
            for (int r = 0; r < 12; ++r)
                for (int c = 0; c < 12; ++c) tr = c_add(tr, c_mul(A[r][c], B[c][r]));
            site_val[16 * s + n] = tr;
        }
    }
}

int32_t or_meson(const int32_t d[4], const double* S1, const double* S2, double* out) {
    const int64_t V = volume(d);
    const int32_t Lt = d[3];
    const int64_t Vs = V / Lt;
    cplx* site_val = (cplx*)malloc(sizeof(cplx) * 16 * (size_t)V);
    if (!site_val) return -1;
    meson_site_values(d, S1, S2, site_val);

    /* Time-slice sums: sequential FP64 over lexicographic sites of each slice. */
    for (int n = 0; n < 16; ++n)
        for (int32_t t = 0; t < Lt; ++t) {
            cplx acc = c_make(0.0, 0.0);
            for (int64_t k = 0; k < Vs; ++k) acc = c_add(acc, site_val[16 * (t * Vs + k) + n]);
            out[2 * (n * Lt + t)] = acc.re;
            out[2 * (n * Lt + t) + 1] = acc.im;
        }
    free(site_val);
    return 0;
}

/* Momentum-projected meson correlators: the same traces weighted by the     */
/* plane wave exp(-i p.x) before the time-slice sum,                         */
/*   C_n(p, t) = sum_{x : x_3 = t} exp(-i p.x) Tr[...],  p_i = 2 pi k_i / L_i */
/* with x the absolute spatial coordinate.  moms holds nmom integer triples  */
/* (k_0, k_1, k_2); out is [nmom][16][Lt][re, im].                           */
int32_t or_meson_mom(const int32_t d[4], const double* S1, const double* S2, int32_t nmom, const int32_t* moms,
                     double* out) {
    const int64_t V = volume(d);
    const int32_t Lt = d[3];
    const int64_t Vs = V / Lt;
    const double two_pi = 6.283185307179586476925286766559;
    cplx* site_val = (cplx*)malloc(sizeof(cplx) * 16 * (size_t)V);
    if (!site_val) return -1;
    meson_site_values(d, S1, S2, site_val);
    for (int32_t q = 0; q < nmom; ++q) {
        const int32_t* k = moms + 3 * q;
        for (int n = 0; n < 16; ++n)
            for (int32_t t = 0; t < Lt; ++t) {
                cplx acc = c_make(0.0, 0.0);
                for (int64_t r = 0; r < Vs; ++r) {
                    const int64_t x = r % d[0], y = (r / d[0]) % d[1], z = r / ((int64_t)d[0] * d[1]);
                    const double px = two_pi * ((double)k[0] * x / d[0] + (double)k[1] * y / d[1] +
                                                (double)k[2] * z / d[2]);
                    acc = c_add(acc, c_mul(c_make(cos(px), -sin(px)), site_val[16 * (t * Vs + r) + n]));
                }
                out[2 * ((q * 16 + n) * Lt + t)] = acc.re;
                out[2 * ((q * 16 + n) * Lt + t) + 1] = acc.im;
            }
    }
    free(site_val);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Nucleon two-point function (the baryon part of the hadron spectrum).      */
/*                                                                           */
/* Interpolators (proton, u u d):                                            */
/*   chi_g(x)     = eps_{abc} (Cg5)_{rs} u^a_r(x) d^b_s(x) u^c_g(x)          */
/*   chibar_g'(0) = eps_{a'b'c'} ubar^{c'}_g' dbar^{b'}_s' G'_{s'r'} ubar^{a'}_r' */
/* with C = gamma_2 gamma_4 (so C gamma_mu C^-1 = -gamma_mu^T) and           */
/* G' = gamma_4 (Cg5)^dagger gamma_4^T = -Cg5, which makes chibar the Dirac  */
/* adjoint of chi.  With S = <q qbar> (S_u = U, S_d = D; sink (spin,colour)  */
/* rows, source columns) Wick's theorem gives a direct and an exchange term  */
/*   <chi_g chibar_g'> = eps eps' (Cg5)_{rs} G'_{s'r'} D^{bb'}_{ss'}         */
/*        [ U^{aa'}_{rr'} U^{cc'}_{gg'} - U^{ac'}_{rg'} U^{ca'}_{gr'} ],     */
/* projected with P = (1 + sign gamma_4)/2: C(t) = sum_{x:x_3=t}             */
/* sum_{g g'} P_{g'g} <chi_g(x) chibar_g'(0)>.  Written with M^{bb'} =       */
/* Cg5 D^{bb'} G' this is                                                    */
/*   eps eps' { Tr[P U^{cc'}] sum_{rr'} U^{aa'}_{rr'} M_{rr'}                */
/*              - sum_{rr'} (U^{ac'} P U^{ca'})_{rr'} M_{rr'} }.             */
/* out is [Lt][re, im].                                                      */
/* ------------------------------------------------------------------------ */

/* Spin block X^{ab}_{rr'} = S[(r a),(r' b)] of a propagator at site s. */
static void spin_block(const double* S, int64_t V, int64_t s, int a, int b, cplx X[4][4]) {
    for (int r = 0; r < 4; ++r)
        for (int rp = 0; rp < 4; ++rp) X[r][rp] = prop_elem(S, V, s, 3 * r + a, 3 * rp + b);
}

int32_t or_nucleon(const int32_t d[4], const double* Su, const double* Sd, int32_t parity, double* out) {
    const int64_t V = volume(d);
    const int32_t Lt = d[3];
    const int64_t Vs = V / Lt;
    static const int perms[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}, {0, 2, 1}, {2, 1, 0}, {1, 0, 2}};
    static const double psign[6] = {1, 1, 1, -1, -1, -1};
    cplx g2[4][4], g4[4][4], g5[4][4], Cm[4][4], Cg5[4][4], Gp[4][4], P[4][4];
    gamma_n(2, g2);
    gamma_n(8, g4);
    gamma_n(15, g5);
    mat4_mul(g2, g4, Cm);
    mat4_mul(Cm, g5, Cg5);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            Gp[i][j] = c_scale(-1.0, Cg5[i][j]);
            P[i][j] = c_scale(0.5 * parity, g4[i][j]);
            if (i == j) P[i][j].re += 0.5;
        }
    cplx* site_val = (cplx*)malloc(sizeof(cplx) * (size_t)V);
    if (!site_val) return -1;

#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        cplx U[3][3][4][4], D[3][3][4][4];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                spin_block(Su, V, s, a, b, U[a][b]);
                spin_block(Sd, V, s, a, b, D[a][b]);
            }
        cplx total = c_make(0.0, 0.0);
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                const int a = perms[i][0], b = perms[i][1], c = perms[i][2];
                const int ap = perms[j][0], bp = perms[j][1], cp = perms[j][2];
                const double sg = psign[i] * psign[j];
                cplx T[4][4], M[4][4], PU[4][4], W[4][4];
                mat4_mul(Cg5, D[b][bp], T);
                mat4_mul(T, Gp, M);
                cplx trPU = c_make(0.0, 0.0);
                mat4_mul(P, U[c][cp], PU);
                for (int r = 0; r < 4; ++r) trPU = c_add(trPU, PU[r][r]);
                mat4_mul(U[a][cp], P, T);
                mat4_mul(T, U[c][ap], W);
                cplx direct = c_make(0.0, 0.0), exch = c_make(0.0, 0.0);
                for (int r = 0; r < 4; ++r)
                    for (int rp = 0; rp < 4; ++rp) {
                        direct = c_add(direct, c_mul(U[a][ap][r][rp], M[r][rp]));
                        exch = c_add(exch, c_mul(W[r][rp], M[r][rp]));
                    }
                const cplx term = c_add(c_mul(trPU, direct), c_scale(-1.0, exch));
                total = c_add(total, c_scale(sg, term));
            }
        site_val[s] = total;
    }
    for (int32_t t = 0; t < Lt; ++t) {
        cplx acc = c_make(0.0, 0.0);
        for (int64_t k = 0; k < Vs; ++k) acc = c_add(acc, site_val[t * Vs + k]);
        out[2 * t] = acc.re;
        out[2 * t + 1] = acc.im;
    }
    free(site_val);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Delta++ two-point function (three identical quarks, u u u).               */
/*                                                                           */
/*   chi^mu_g(x)     = eps_{abc} (C gamma_mu)_{rs} u^a_r u^b_s u^c_g          */
/*   chibar^mu_g'(0) = eps_{a'b'c'} ubar^{c'}_g' ubar^{b'}_s' G'_{s'r'} ubar^{a'}_r' */
/* with G' = gamma_4 (C gamma_mu)^dagger gamma_4^T (the Dirac adjoint) and   */
/* C = gamma_2 gamma_4.  With q1 = (a r), q2 = (b s), q3 = (c g) at the sink */
/* and q1' = (a' r'), q2' = (b' s'), q3' = (c' g') at the source, Wick's     */
/* theorem gives <q1 q2 q3 qbar3' qbar2' qbar1'> = det_{ij} S(q_i, q_j'), the */
/* identity pairing counted +.  The result, projected with                   */
/* P = (1 + parity gamma_4)/2 and summed over the spatial mu = 1, 2, 3, is   */
/*   C(t) = sum_{x: x_3 = t} sum_mu sum_{g g'} P_{g'g} <chi^mu_g chibar^mu_g'>. */
/* Written with dense 4x4 matrices and plain loops.  out is [Lt][re, im].     */
/* ------------------------------------------------------------------------ */

int32_t or_delta(const int32_t d[4], const double* S, int32_t parity, double* out) {
    const int64_t V = volume(d);
    const int32_t Lt = d[3];
    const int64_t Vs = V / Lt;
    static const int perms[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}, {0, 2, 1}, {2, 1, 0}, {1, 0, 2}};
    static const double psign[6] = {1, 1, 1, -1, -1, -1};
    cplx g[5][4][4], Cm[4][4], G[3][4][4], Gp[3][4][4], P[4][4], T[4][4];
    gamma_n(1, g[1]);
    gamma_n(2, g[2]);
    gamma_n(4, g[3]);
    gamma_n(8, g[4]);
    mat4_mul(g[2], g[4], Cm);
    for (int mu = 0; mu < 3; ++mu) {
        mat4_mul(Cm, g[mu + 1], G[mu]);
        /* G' = gamma_4 G^dagger gamma_4^T */
        cplx Gd[4][4], g4t[4][4];
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                Gd[i][j] = c_conj(G[mu][j][i]);
                g4t[i][j] = g[4][j][i];
            }
        mat4_mul(g[4], Gd, T);
        mat4_mul(T, g4t, Gp[mu]);
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            P[i][j] = c_scale(0.5 * parity, g[4][i][j]);
            if (i == j) P[i][j].re += 0.5;
        }
    cplx* site_val = (cplx*)malloc(sizeof(cplx) * (size_t)V);
    if (!site_val) return -1;

#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        cplx total = c_make(0.0, 0.0);
        for (int mu = 0; mu < 3; ++mu)
            for (int i = 0; i < 6; ++i)
                for (int j = 0; j < 6; ++j) {
                    const int a = perms[i][0], b = perms[i][1], c = perms[i][2];
                    const int ap = perms[j][0], bp = perms[j][1], cp = perms[j][2];
                    const double sg = psign[i] * psign[j];
                    for (int r = 0; r < 4; ++r)
                        for (int sp = 0; sp < 4; ++sp) {
                            const cplx gs = G[mu][r][sp];
                            if (gs.re == 0.0 && gs.im == 0.0) continue;
                            for (int spp = 0; spp < 4; ++spp)
                                for (int rp = 0; rp < 4; ++rp) {
                                    const cplx gps = Gp[mu][spp][rp];
                                    if (gps.re == 0.0 && gps.im == 0.0) continue;
                                    for (int gm = 0; gm < 4; ++gm)
                                        for (int gmp = 0; gmp < 4; ++gmp) {
                                            const cplx pp = P[gmp][gm];
                                            if (pp.re == 0.0 && pp.im == 0.0) continue;
                                            /* rows: sink quarks (a r), (b sp), (c gm);
                                               columns: source quarks (a' rp), (b' spp), (c' gmp) */
                                            const int row[3] = {3 * r + a, 3 * sp + b, 3 * gm + c};
                                            const int col[3] = {3 * rp + ap, 3 * spp + bp, 3 * gmp + cp};
                                            cplx m[3][3];
                                            for (int x = 0; x < 3; ++x)
                                                for (int y = 0; y < 3; ++y) m[x][y] = prop_elem(S, V, s, row[x], col[y]);
                                            const cplx det = c_add(
                                                c_add(c_mul(m[0][0], c_add(c_mul(m[1][1], m[2][2]),
                                                                          c_scale(-1.0, c_mul(m[1][2], m[2][1])))),
                                                      c_scale(-1.0, c_mul(m[0][1], c_add(c_mul(m[1][0], m[2][2]),
                                                                                         c_scale(-1.0, c_mul(m[1][2], m[2][0])))))),
                                                c_mul(m[0][2], c_add(c_mul(m[1][0], m[2][1]),
                                                                     c_scale(-1.0, c_mul(m[1][1], m[2][0])))));
                                            const cplx coef = c_mul(c_mul(gs, gps), pp);
                                            total = c_add(total, c_scale(sg, c_mul(coef, det)));
                                        }
                                }
                        }
                }
        site_val[s] = total;
    }
    for (int32_t t = 0; t < Lt; ++t) {
        cplx acc = c_make(0.0, 0.0);
        for (int64_t k = 0; k < Vs; ++k) acc = c_add(acc, site_val[t * Vs + k]);
        out[2 * t] = acc.re;
        out[2 * t + 1] = acc.im;
    }
    free(site_val);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sums (global and time-slice), FP64, sequential over lexicographic sites.  */
/* ------------------------------------------------------------------------ */

/* out[t][k] = sum over sites of slice t of component k (complex), for a field
 * of ncomplex complex numbers per site; out is [Lt][ncomplex][re, im]. */
void or_timeslice_sum(const int32_t d[4], int32_t ncomplex, const double* f, double* out) {
    const int64_t V = volume(d);
    const int32_t Lt = d[3];
    const int64_t Vs = V / Lt;
    for (int32_t t = 0; t < Lt; ++t)
        for (int32_t k = 0; k < ncomplex; ++k) {
            double re = 0.0, im = 0.0;
            for (int64_t x = 0; x < Vs; ++x) {
                const double* p = f + 2 * ((t * Vs + x) * ncomplex + k);
                re += p[0];
                im += p[1];
            }
            out[2 * (t * ncomplex + k)] = re;
            out[2 * (t * ncomplex + k) + 1] = im;
        }
}

/* sum_x |f(x)|^2 over all components */
double or_norm2(int64_t n_complex_total, const double* f) {
    double acc = 0.0;
    for (int64_t i = 0; i < n_complex_total; ++i)
        acc += f[2 * i] * f[2 * i] + f[2 * i + 1] * f[2 * i + 1];
    return acc;
}

/* sum_x conj(a(x)) . b(x) over all components; out = (re, im) */
void or_inner(int64_t n_complex_total, const double* a, const double* b, double* out) {
    cplx acc = c_make(0.0, 0.0);
    for (int64_t i = 0; i < n_complex_total; ++i) {
        const cplx x = c_make(a[2 * i], a[2 * i + 1]);
        const cplx y = c_make(b[2 * i], b[2 * i + 1]);
        acc = c_add(acc, c_mul(c_conj(x), y));
    }
    out[0] = acc.re;
    out[1] = acc.im;
}
