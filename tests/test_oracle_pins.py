"""Pins of the FP64 oracle against facts fixed by the mathematics.

Each test checks the oracle against something other than itself: Fourier
closed forms, exact rationals, gauge symmetry, Hermiticity, locality, a dense
brute-force operator on a 2^4 lattice, the Clifford algebra, Fierz
completeness and gamma_5 hermiticity.  Smearing operator reading:
(1 + kappa H)^N with H the gauge-covariant spatial hopping term; its
unit-gauge eigenvalues are 1 + 2 kappa sum_i cos p_i.
"""


import numpy as np
import pytest

import oracle
from paper_1111_5596_amd import synth


def unit_links(dims):
    V = synth.volume(dims)
    U = np.zeros((4, V, 3, 3), dtype=np.complex128)
    U[:] = np.eye(3)
    return U


def fourier_smear(dims, psi, kappa, n):
    """(1 + kappa H)^n for unit links via the eigenvalues of the spatial
    hopping term: plane waves, lambda(p) = 1 + 2 kappa sum_i cos p_i."""
    Lx, Ly, Lz, Lt = dims
    a = psi.reshape(Lt, Lz, Ly, Lx, -1)
    f = np.fft.fftn(a, axes=(1, 2, 3))
    pz = 2 * np.pi * np.arange(Lz) / Lz
    py = 2 * np.pi * np.arange(Ly) / Ly
    px = 2 * np.pi * np.arange(Lx) / Lx
    lam = 1 + 2 * kappa * (np.cos(pz)[:, None, None] + np.cos(py)[None, :, None]
                           + np.cos(px)[None, None, :])
    f = f * (lam ** n)[None, :, :, :, None]
    return np.fft.ifftn(f, axes=(1, 2, 3)).reshape(psi.shape)


def gauge_rotate_links(dims, U, g):
    """U^g_mu(x) = g(x) U_mu(x) g(x + mu)^dagger."""
    out = np.empty_like(U)
    for mu in range(4):
        g_fwd = oracle.shift(g, dims, mu, +1)
        out[mu] = np.einsum("vab,vbc,vdc->vad", g, U[mu], np.conj(g_fwd))
    return out


def gauge_rotate_fermions(g, psi):
    return np.einsum("vab,...vsb->...vsa", g, psi)


# --------------------------------------------------------------------------
# Geometry and shift (pins P6)
# --------------------------------------------------------------------------

def test_neighbour_wraps_periodically():
    dims = (4, 6, 2, 8)
    V = synth.volume(dims)
    for s in [0, 3, 5, V - 1, 77]:
        x = [s % 4, (s // 4) % 6, (s // 24) % 2, s // 48]
        for mu in range(4):
            for step in (+1, -1):
                y = list(x)
                y[mu] = (y[mu] + step) % dims[mu]
                expect = y[0] + 4 * (y[1] + 6 * (y[2] + 2 * y[3]))
                assert oracle.neighbour(dims, s, mu, step) == expect


def test_shift_identities_bitwise():
    dims = (4, 6, 2, 8)
    rng = np.random.default_rng(0)
    V = synth.volume(dims)
    f = rng.normal(size=(V, 4, 3)) + 1j * rng.normal(size=(V, 4, 3))
    for mu in range(4):
        back = oracle.shift(oracle.shift(f, dims, mu, +1), dims, mu, -1)
        assert np.array_equal(back, f)
        g = f
        for _ in range(dims[mu]):
            g = oracle.shift(g, dims, mu, +1)
        assert np.array_equal(g, f)


def test_shift_matches_array_roll():
    """shift(f, +mu)(x) = f(x + mu): compare with numpy's roll of the 4-D array."""
    dims = (4, 6, 2, 8)
    V = synth.volume(dims)
    f = np.arange(V, dtype=np.float64).astype(np.complex128)
    a = f.reshape(8, 2, 6, 4)
    for mu, axis in zip(range(4), (3, 2, 1, 0)):
        for sign in (+1, -1):
            expect = np.roll(a, -sign, axis=axis).reshape(-1)
            assert np.array_equal(oracle.shift(f, dims, mu, sign), expect)


# --------------------------------------------------------------------------
# Smearing: free field (P1, P2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dims,n", [((4, 4, 4, 8), 10), ((2, 2, 2, 2), 10),
                                    ((6, 4, 8, 2), 7), ((8, 8, 8, 2), 25)])
def test_free_field_fourier_closed_form(dims, n):
    kappa = 0.25
    U = unit_links(dims)
    src = synth.point_source(dims, [0, 7])
    got = oracle.smear(U, src, dims, kappa, n)
    for c in range(2):
        expect = fourier_smear(dims, src[c].reshape(-1, 12), kappa, n).reshape(src[c].shape)
        scale = np.abs(expect).max()
        assert np.abs(got[c] - expect).max() <= 1e-13 * scale


def test_free_field_random_source_fourier():
    dims = (6, 4, 2, 3)
    rng = np.random.default_rng(5)
    V = synth.volume(dims)
    psi = rng.normal(size=(1, V, 4, 3)) + 1j * rng.normal(size=(1, V, 4, 3))
    got = oracle.smear(unit_links(dims), psi, dims, 0.13, 9)
    expect = fourier_smear(dims, psi[0].reshape(V, 12), 0.13, 9).reshape(V, 4, 3)
    assert np.abs(got[0] - expect).max() <= 1e-12 * np.abs(expect).max()


def test_free_field_printed_values_4cubed():
    """Unit links, point source, kappa = 1/4, N = 10 on 4^3 x 8: every value is
    an integer over 4^10 and FP64 holds it exactly.  The sum over sites is
    (1 + 6 kappa)^N (zero-momentum eigenvalue) and the sum of squares follows
    from Parseval."""
    dims = (4, 4, 4, 8)
    out = oracle.smear(unit_links(dims), synth.point_source(dims, [0]), dims, 0.25, 10)[0]
    phi = out[:, 0, 0]
    assert phi.sum() == 2.5 ** 10  # 9536.7431640625 exactly
    scaled = phi.real * 4 ** 10
    assert np.array_equal(scaled, np.round(scaled))
    assert np.all(phi.imag == 0)
    # Parseval: sum |phi|^2 = Vs^-1 sum_p lambda(p)^(2N)
    p = 2 * np.pi * np.arange(4) / 4
    lam = 1 + 0.5 * (np.cos(p)[:, None, None] + np.cos(p)[None, :, None] + np.cos(p)[None, None, :])
    parseval = np.sum(lam ** 20) / 64
    assert abs(np.sum(np.abs(phi) ** 2) - parseval) <= 1e-12 * parseval
    # the other 11 spin-colour components stay exactly zero
    assert np.count_nonzero(out[:, 1:, :]) == 0 and np.count_nonzero(out[:, 0, 1:]) == 0


def test_free_field_exact_walk_count():
    """kappa = 1/4: 4^N psi_N(x) counts weighted lattice walks; computed here in
    exact integer arithmetic by repeated neighbour addition on a 3x5x2 slice."""
    dims = (3, 5, 2, 1)
    n = 6
    Lx, Ly, Lz, _ = dims
    cnt = np.zeros((Lz, Ly, Lx), dtype=object)
    cnt[0, 0, 0] = 1
    for _ in range(n):
        new = cnt * 4  # 4^k psi_k: the identity term carries the factor 4
        for axis in range(3):
            new = new + np.roll(cnt, 1, axis=axis) + np.roll(cnt, -1, axis=axis)
        cnt = new
    got = oracle.smear(unit_links(dims), synth.point_source(dims, [0]), dims, 0.25, n)[0]
    expect = np.array([float(v) for v in cnt.reshape(-1)]) / 4 ** n
    assert np.array_equal(got[:, 0, 0].real, expect)


# --------------------------------------------------------------------------
# Smearing: gauge covariance, Hermiticity, linearity, locality (P3, P8, P9)
# --------------------------------------------------------------------------

def test_gauge_covariance():
    dims = (4, 4, 4, 8)
    U = synth.su3_links(dims, 1)
    psi = synth.gaussian_propagator(dims, 101, ncols=3)
    g = synth.gauge_transform(dims, 9001)
    lhs = oracle.smear(gauge_rotate_links(dims, U, g), gauge_rotate_fermions(g, psi), dims, 0.25, 10)
    rhs = gauge_rotate_fermions(g, oracle.smear(U, psi, dims, 0.25, 10))
    assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(rhs)


def test_gauge_covariance_detects_wrong_link():
    """Sanity of the pin itself: a hop that uses U_mu(x) on the backward
    neighbour is not covariant, and the test above would catch it."""
    dims = (4, 4, 2, 2)
    U = synth.su3_links(dims, 2)
    psi = synth.gaussian_propagator(dims, 102, ncols=1)[0]
    g = synth.gauge_transform(dims, 9002)

    def wrong_step(U, psi):
        out = psi.copy()
        for i in range(3):
            out += 0.25 * np.einsum("vab,vsb->vsa", U[i], oracle.shift(psi, dims, i, +1))
            out += 0.25 * np.einsum("vba,vsb->vsa", np.conj(U[i]), oracle.shift(psi, dims, i, -1))
        return out

    Ug = gauge_rotate_links(dims, U, g)
    lhs = wrong_step(Ug, gauge_rotate_fermions(g, psi))
    rhs = gauge_rotate_fermions(g, wrong_step(U, psi))
    assert np.linalg.norm(lhs - rhs) > 1e-3 * np.linalg.norm(rhs)


def test_hermiticity_and_linearity():
    dims = (4, 2, 6, 3)
    U = synth.su3_links(dims, 7)
    a = synth.gaussian_propagator(dims, 11, ncols=1)[0]
    b = synth.gaussian_propagator(dims, 12, ncols=1)[0]
    Ma = oracle.smear_step(U, a, dims, 0.21)
    Mb = oracle.smear_step(U, b, dims, 0.21)
    lhs = np.vdot(b, Ma)
    rhs = np.vdot(Mb, a)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    alpha, beta = 0.3 - 1.1j, 2.0 + 0.5j
    comb = oracle.smear(U, alpha * a + beta * b, dims, 0.21, 4)[0]
    sep = alpha * oracle.smear(U, a, dims, 0.21, 4)[0] + beta * oracle.smear(U, b, dims, 0.21, 4)[0]
    assert np.linalg.norm(comb - sep) <= 1e-13 * np.linalg.norm(sep)


def test_time_slice_locality():
    dims = (4, 4, 4, 8)
    U = synth.su3_links(dims, 1)
    t0 = 3
    src = synth.point_source(dims, range(12), site=t0 * 64 + 5)
    out = oracle.smear(U, src, dims, 0.25, 10)
    per_slice = np.abs(out).reshape(12, 8, 64, 12).sum(axis=(0, 2, 3))
    assert per_slice[t0] > 0
    assert np.count_nonzero(per_slice[np.arange(8) != t0]) == 0


# --------------------------------------------------------------------------
# Dense brute force on the 2^4 lattice (P7)
# --------------------------------------------------------------------------

def dense_operator(dims, U, kappa):
    """192x192 matrix 1 + kappa H built by enumerating every (site, spatial
    direction, sign) hop; hops that land on the same site add up."""
    V = synth.volume(dims)
    n = 12 * V
    M = np.eye(n, dtype=np.complex128)

    def coords(s):
        return [s % dims[0], (s // dims[0]) % dims[1], (s // (dims[0] * dims[1])) % dims[2],
                s // (dims[0] * dims[1] * dims[2])]

    def index(c):
        return c[0] + dims[0] * (c[1] + dims[1] * (c[2] + dims[2] * c[3]))

    for s in range(V):
        c = coords(s)
        for i in range(3):
            for sign in (+1, -1):
                d = list(c)
                d[i] = (d[i] + sign) % dims[i]
                y = index(d)
                link = U[i, s] if sign > 0 else np.conj(U[i, y]).T
                for spin in range(4):
                    rows = 12 * s + 3 * spin + np.arange(3)
                    cols = 12 * y + 3 * spin + np.arange(3)
                    M[np.ix_(rows, cols)] += kappa * link
    return M


def test_brute_force_2to4_smearing():
    dims = (2, 2, 2, 2)
    U = synth.su3_links(dims, 44)
    M = dense_operator(dims, U, 0.25)
    MN = np.linalg.matrix_power(M, 10)
    src = synth.point_source(dims, range(12))
    got = oracle.smear(U, src, dims, 0.25, 10)
    for j in range(12):
        expect = MN @ src[j].reshape(-1)
        assert np.abs(got[j].reshape(-1) - expect).max() <= 1e-13 * np.abs(expect).max()


def test_brute_force_2to4_contraction():
    """Contraction via explicit 12x12 matrices and Kronecker products."""
    dims = (2, 2, 2, 2)
    S1 = synth.gaussian_propagator(dims, 45)
    S2 = synth.gaussian_propagator(dims, 46)
    got = oracle.meson(S1, S2, dims)
    V = 16
    g5 = np.kron(oracle.gamma(15), np.eye(3))
    expect = np.zeros((16, 2), dtype=np.complex128)
    for n in range(16):
        G = np.kron(oracle.gamma(n), np.eye(3))
        for s in range(V):
            A = S1[:, s].reshape(12, 12).T  # rows sink (spin, colour), cols source j
            B = S2[:, s].reshape(12, 12).T
            expect[n, s // 8] += np.trace(g5 @ B.conj().T @ g5 @ G @ A @ G)
    assert np.abs(got - expect).max() <= 1e-13 * np.abs(expect).max()


# --------------------------------------------------------------------------
# Gamma matrices (P11)
# --------------------------------------------------------------------------

def test_gamma_clifford_and_gamma5():
    g = [oracle.gamma(1 << k) for k in range(4)]
    for a in range(4):
        assert np.allclose(g[a], g[a].conj().T, atol=0)
        for b in range(4):
            anti = g[a] @ g[b] + g[b] @ g[a]
            assert np.array_equal(anti, 2 * np.eye(4) * (a == b))
    assert np.array_equal(oracle.gamma(15), np.diag([1, 1, -1, -1]).astype(complex))
    assert np.array_equal(oracle.gamma(0), np.eye(4, dtype=complex))
    # gamma_4 in the DeGrand-Rossi basis couples upper and lower spin pairs
    assert np.array_equal(np.abs(oracle.gamma(8)), np.kron([[0, 1], [1, 0]], np.eye(2)))


def test_gamma_signed_permutations_klein_group():
    klein = {(0, 1, 2, 3), (1, 0, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)}
    groups = {}
    for n in range(16):
        G = oracle.gamma(n)
        perm = tuple(int(np.flatnonzero(G[r])[0]) for r in range(4))
        assert all(np.count_nonzero(G[r]) == 1 for r in range(4))
        assert perm in klein
        assert all(abs(G[r, perm[r]]) == 1 for r in range(4))
        groups.setdefault(perm, []).append(n)
    assert sorted(map(tuple, groups.values())) == [(0, 3, 12, 15), (1, 2, 13, 14),
                                                   (4, 7, 8, 11), (5, 6, 9, 10)]


def test_gamma_squares():
    for n in range(16):
        k = bin(n).count("1")
        eps = (-1) ** (k * (k - 1) // 2)
        G = oracle.gamma(n)
        assert np.array_equal(G @ G, eps * np.eye(4))


# --------------------------------------------------------------------------
# Contraction (P4, P10, Fierz completeness)
# --------------------------------------------------------------------------

def _epsilon(n):
    k = bin(n).count("1")
    return (-1) ** (k * (k - 1) // 2)


def _spin_trace(S):
    """(Tr_spin S)(x)_{ab} = sum_alpha S[(alpha a), (alpha b)], (V, 3, 3)."""
    V = S.shape[1]
    out = np.zeros((V, 3, 3), dtype=np.complex128)
    for alpha in range(4):
        for b in range(3):
            out[:, :, b] += S[3 * alpha + b, :, alpha, :]
    return out


def test_contraction_gamma5_hermiticity_and_bounds():
    dims = (4, 4, 2, 6)
    S = synth.gaussian_propagator(dims, 33)
    C = oracle.meson(S, S, dims)
    per_site = np.sum(np.abs(S) ** 2, axis=(0, 2, 3)).reshape(6, -1).sum(axis=1)
    assert np.abs(C[15] - per_site).max() <= 1e-13 * per_site.max()
    assert np.abs(C.imag).max() <= 1e-13 * per_site.max()
    assert np.all(np.abs(C) <= C[15].real[None, :] * (1 + 1e-13))
    assert abs(C[15].sum() - np.sum(np.abs(S) ** 2)) <= 1e-13 * np.sum(np.abs(S) ** 2)


def test_contraction_fierz_completeness():
    """sum_n eps_n Gamma_n A Gamma_n = 4 Tr(A) 1  (eps_n = Gamma_n^2), so
    sum_n eps_n C_n(t) = 4 sum_{x in t} Tr_c[(Tr_s S2)^dagger (Tr_s S1)]."""
    dims = (2, 4, 2, 3)
    S1 = synth.gaussian_propagator(dims, 51)
    S2 = synth.gaussian_propagator(dims, 52)
    C = oracle.meson(S1, S2, dims)
    lhs = sum(_epsilon(n) * C[n] for n in range(16))
    T1, T2 = _spin_trace(S1), _spin_trace(S2)
    site = 4 * np.einsum("vab,vab->v", np.conj(T2), T1)
    rhs = site.reshape(3, -1).sum(axis=1)
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(rhs).max()


def test_contraction_gauge_invariance():
    dims = (4, 4, 4, 4)
    S1 = synth.gaussian_propagator(dims, 61)
    S2 = synth.gaussian_propagator(dims, 62)
    g = synth.gauge_transform(dims, 9003)
    C = oracle.meson(S1, S2, dims)
    Cg = oracle.meson(gauge_rotate_fermions(g, S1), gauge_rotate_fermions(g, S2), dims)
    assert np.abs(C - Cg).max() <= 1e-13 * np.abs(C).max()


def test_free_point_source_correlator_closed_form():
    """Unit links, 12-column point source: S(x) = phi(x) 1_12 with phi the
    free smeared scalar, so C_n(t0) = 12 eps_n sum_x phi(x)^2 and C_n(t) = 0
    elsewhere; sum phi^2 comes from Parseval."""
    dims = (4, 4, 4, 8)
    S = oracle.smear(unit_links(dims), synth.point_source(dims, range(12)), dims, 0.25, 6)
    C = oracle.meson(S, S, dims)
    p = 2 * np.pi * np.arange(4) / 4
    lam = 1 + 0.5 * (np.cos(p)[:, None, None] + np.cos(p)[None, :, None] + np.cos(p)[None, None, :])
    sum_phi2 = np.sum(lam ** 12) / 64
    for n in range(16):
        assert abs(C[n, 0] - 12 * _epsilon(n) * sum_phi2) <= 1e-12 * sum_phi2
        assert np.count_nonzero(C[n, 1:]) == 0


# --------------------------------------------------------------------------
# Momentum-projected contraction
# --------------------------------------------------------------------------

def test_momentum_free_point_source_convolution():
    """Unit links, 12-column point source: S(x) = phi(x) 1_12, so
    C_n(p, t0) = 12 eps_n sum_x exp(-i p.x) phi(x)^2, which by the
    convolution theorem is 12 eps_n Vs^-1 sum_q lambda(q)^N lambda(q - p)^N;
    the momentum sum is over the Brillouin zone, not over sites."""
    dims = (4, 6, 2, 4)
    N = 5
    S = oracle.smear(unit_links(dims), synth.point_source(dims, range(12)), dims, 0.25, N)
    moms = [(0, 0, 0), (1, 0, 0), (0, 2, 1), (3, 5, 1), (-1, 1, 0)]
    C = oracle.meson_mom(S, S, dims, moms)
    L = dims[:3]
    q = [2 * np.pi * np.arange(l) / l for l in L]
    Q = np.meshgrid(*q, indexing="ij")
    lam = 1 + 0.5 * (np.cos(Q[0]) + np.cos(Q[1]) + np.cos(Q[2]))
    Vs = L[0] * L[1] * L[2]
    for m, k in enumerate(moms):
        shifted = np.roll(lam, shift=k, axis=(0, 1, 2))  # lambda(q - p)
        expect = np.sum(lam ** N * shifted ** N) / Vs
        for n in range(16):
            assert abs(C[m, n, 0] - 12 * _epsilon(n) * expect) <= 1e-12 * lam.max() ** (2 * N)
            assert np.count_nonzero(C[m, n, 1:]) == 0


def test_momentum_zero_is_the_plain_correlator_and_translation_phase():
    """p = 0 gives C_n(t); translating both propagators by a spatial vector d
    multiplies C_n(p, t) by exp(-i p.d)."""
    dims = (4, 2, 6, 3)
    U = synth.su3_links(dims, 61)
    S1 = oracle.smear(U, synth.gaussian_propagator(dims, 161), dims, 0.2, 3)
    S2 = synth.gaussian_propagator(dims, 162)
    moms = [(0, 0, 0), (1, 1, 1), (2, 0, -1), (-1, 1, 5)]
    C = oracle.meson_mom(S1, S2, dims, moms)
    C0 = oracle.meson(S1, S2, dims)
    assert np.abs(C[0] - C0).max() <= 1e-14 * np.abs(C0).max()
    d = (1, 1, 2)

    def translate(S):  # S'(x) = S(x - d), column by column
        out = []
        for col in S:
            for mu in range(3):
                for _ in range(d[mu]):
                    col = oracle.shift(col, dims, mu, -1)
            out.append(col)
        return np.stack(out)

    Ct = oracle.meson_mom(translate(S1), translate(S2), dims, moms)
    for m, k in enumerate(moms):
        phase = np.exp(-2j * np.pi * sum(k[i] * d[i] / dims[i] for i in range(3)))
        assert np.abs(Ct[m] - phase * C[m]).max() <= 1e-12 * np.abs(C0).max()


def test_momentum_inverse_transform_recovers_the_origin():
    """Summing C_n(p, t) over the whole Brillouin zone gives Vs times the
    trace at the spatial origin of slice t (here read off by contracting
    propagators that vanish everywhere else)."""
    dims = (2, 4, 2, 3)
    S1 = synth.gaussian_propagator(dims, 171)
    S2 = synth.gaussian_propagator(dims, 172)
    moms = [(a, b, c) for a in range(2) for b in range(4) for c in range(2)]
    Csum = oracle.meson_mom(S1, S2, dims, moms).sum(axis=0)
    Vs = 16
    origin = np.zeros(synth.volume(dims), dtype=bool)
    origin[np.arange(dims[3]) * Vs] = True
    C_origin = oracle.meson(S1 * origin[None, :, None, None], S2 * origin[None, :, None, None], dims)
    assert np.abs(Csum - Vs * C_origin).max() <= 1e-12 * np.abs(Csum).max()


# --------------------------------------------------------------------------
# Nucleon two-point function
# --------------------------------------------------------------------------

# DeGrand-Rossi gamma_1..gamma_4 written out (independent of the oracle's tables)
_DR = [np.array(m, dtype=np.complex128) for m in (
    [[0, 0, 0, 1j], [0, 0, 1j, 0], [0, -1j, 0, 0], [-1j, 0, 0, 0]],
    [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],
    [[0, 0, 1j, 0], [0, 0, 0, -1j], [-1j, 0, 0, 0], [0, 1j, 0, 0]],
    [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]])]


def _levi_civita():
    eps = np.zeros((3, 3, 3))
    for (a, b, c), sg in [((0, 1, 2), 1), ((1, 2, 0), 1), ((2, 0, 1), 1), ((0, 2, 1), -1), ((2, 1, 0), -1),
                          ((1, 0, 2), -1)]:
        eps[a, b, c] = sg
    return eps


def _nucleon_by_wick(Su, Sd, dims, parity):
    """Proton correlator from the interpolators by Wick's theorem, with no
    factorisation: for chi = eps (u^T Cg5 d) u and chibar its Dirac adjoint,
    <u1 d2 u3 ubar3' dbar2' ubar1'> = D(2,2') det[[U(1,1'), U(1,3')], [U(3,1'), U(3,3')]],
    every index tuple summed with einsum."""
    g1, g2, g3, g4 = _DR
    g5 = g1 @ g2 @ g3 @ g4
    C = g2 @ g4
    assert np.allclose(C @ g1 @ np.linalg.inv(C), -g1.T) and np.allclose(C @ g4 @ np.linalg.inv(C), -g4.T)
    Gsnk = C @ g5
    Gsrc = g4 @ Gsnk.conj().T @ g4.T  # chibar = chi^dagger gamma_4
    P = 0.5 * (np.eye(4) + parity * g4)
    eps = _levi_civita()
    V = synth.volume(dims)
    # U[x, r, a, r', a'] = S[(r a), (r' a')] = component (r, a) of column 3 r' + a'
    U = np.transpose(Su.reshape(4, 3, V, 4, 3), (2, 3, 4, 0, 1))
    D = np.transpose(Sd.reshape(4, 3, V, 4, 3), (2, 3, 4, 0, 1))
    # sink colours a b c, spins r s g; source colours A B C, spins R S G
    direct = np.einsum("abc,rs,ABC,SR,xraRA,xsbSB,xgcGC,Gg->x", eps, Gsnk, eps, Gsrc, U, D, U, P, optimize=True)
    exch = np.einsum("abc,rs,ABC,SR,xraGC,xsbSB,xgcRA,Gg->x", eps, Gsnk, eps, Gsrc, U, D, U, P, optimize=True)
    site = direct - exch
    return site.reshape(dims[3], -1).sum(axis=1)


@pytest.mark.parametrize("parity", [1, -1])
def test_nucleon_matches_unfactorised_wick_contraction(parity):
    dims = (2, 2, 4, 3)
    Su = synth.gaussian_propagator(dims, 181)
    Sd = synth.gaussian_propagator(dims, 182)
    got = oracle.nucleon(Su, Sd, dims, parity)
    ref = _nucleon_by_wick(Su, Sd, dims, parity)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_nucleon_free_point_source_closed_form():
    """Unit links, 12-column point source: S(x) = phi(x) 1_12 and the two
    Wick terms give 48 + 12 = 60 phi(x)^3 for either parity, so
    C(t0) = 60 sum_x phi^3 = 60 Vs^-2 sum_{q1,q2} lambda(q1)^N lambda(q2)^N lambda(q1+q2)^N."""
    dims = (4, 6, 2, 4)
    N = 4
    S = oracle.smear(unit_links(dims), synth.point_source(dims, range(12)), dims, 0.25, N)
    L = dims[:3]
    Q = np.meshgrid(*[2 * np.pi * np.arange(l) / l for l in L], indexing="ij")
    lam = (1 + 0.5 * (np.cos(Q[0]) + np.cos(Q[1]) + np.cos(Q[2]))) ** N
    Vs = L[0] * L[1] * L[2]
    flat = lam.reshape(-1)
    idx = np.indices(L).reshape(3, -1)
    total = 0.0
    for i in range(Vs):  # q1 + q2 mod L
        k = (idx[:, i:i + 1] + idx) % np.array(L)[:, None]
        total += flat[i] * np.sum(flat * lam[k[0], k[1], k[2]])
    expect = 60 * total / Vs ** 2
    for parity in (1, -1):
        C = oracle.nucleon(S, S, dims, parity)
        assert abs(C[0] - expect) <= 1e-12 * expect
        assert np.count_nonzero(C[1:]) == 0


def test_nucleon_gauge_invariance_and_parity_sum():
    """eps eps' is SU(3) invariant: C(t) is unchanged under S(x) -> g(x) S(x);
    the two parity projections add up to the unprojected trace (P = 1),
    which the unfactorised contraction supplies."""
    dims = (4, 2, 2, 3)
    Su = synth.gaussian_propagator(dims, 191)
    Sd = synth.gaussian_propagator(dims, 192)
    g = synth.gauge_transform(dims, 9191)
    C = oracle.nucleon(Su, Sd, dims, 1)
    Cg = oracle.nucleon(gauge_rotate_fermions(g, Su), gauge_rotate_fermions(g, Sd), dims, 1)
    assert np.abs(C - Cg).max() <= 1e-13 * np.abs(C).max()
    Cm = oracle.nucleon(Su, Sd, dims, -1)
    unproj = _nucleon_by_wick(Su, Sd, dims, 1) + _nucleon_by_wick(Su, Sd, dims, -1)
    assert np.abs(C + Cm - unproj).max() <= 1e-13 * np.abs(unproj).max()
    # the pin has teeth: a contraction that used D^{b'b} for D^{bb'} (sink and
    # source colour of d exchanged) is not invariant
    def colour_t(S):
        return np.transpose(S.reshape(4, 3, -1, 4, 3), (0, 4, 2, 3, 1)).reshape(S.shape)

    Ct = oracle.nucleon(Su, colour_t(Sd), dims, 1)
    Ctg = oracle.nucleon(gauge_rotate_fermions(g, Su), colour_t(gauge_rotate_fermions(g, Sd)), dims, 1)
    assert np.abs(Ct - Ctg).max() > 1e-3 * np.abs(Ct).max()


def _delta_gammas(parity):
    g1, g2, g3, g4 = _DR
    C = g2 @ g4
    G = [C @ g for g in (g1, g2, g3)]
    Gp = [g4 @ x.conj().T @ g4.T for x in G]
    P = 0.5 * (np.eye(4) + parity * g4)
    return G, Gp, P


def _delta_by_wick(S, dims, parity):
    """Delta++ correlator as the six Wick terms of <q1 q2 q3 qbar3' qbar2' qbar1'>
    written out one by one (einsum over every index), summed over mu = 1..3."""
    G, Gp, P = _delta_gammas(parity)
    eps = _levi_civita()
    V = synth.volume(dims)
    U = np.transpose(S.reshape(4, 3, V, 4, 3), (2, 3, 4, 0, 1))  # U[x, r, a, R, A]
    # sink quarks (a r), (b s), (c g); source quarks (A R), (B S), (C G)
    terms = [("xraRA,xsbSB,xgcGC", 1), ("xraSB,xsbRA,xgcGC", -1), ("xraGC,xsbSB,xgcRA", -1),
             ("xraRA,xsbGC,xgcSB", -1), ("xraSB,xsbGC,xgcRA", 1), ("xraGC,xsbRA,xgcSB", 1)]
    site = np.zeros(V, dtype=np.complex128)
    for mu in range(3):
        for t, sg in terms:
            site += sg * np.einsum("abc,rs,ABC,SR,Gg," + t + "->x", eps, G[mu], eps, Gp[mu], P, U, U, U,
                                   optimize=True)
    return site.reshape(dims[3], -1).sum(axis=1)


@pytest.mark.parametrize("parity", [1, -1])
def test_delta_matches_wick_terms(parity):
    dims = (2, 2, 2, 3)
    S = synth.gaussian_propagator(dims, 183)
    got = oracle.delta(S, dims, parity)
    ref = _delta_by_wick(S, dims, parity)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_delta_free_point_source_closed_form():
    """Unit links, 12-column point source: S = phi(x) 1_12.  The colour sums
    give 6 for every Wick term, and the spin sums reduce each term to a trace:
    C(t0) = 6 sum_x phi^3 sum_mu [Tr(G G') Tr P + Tr(G G'^T) Tr P + Tr(G G' P^T)
    + Tr(G P G') + Tr(G P G'^T) + Tr(G G'^T P^T)], with sum_x phi^3 from the
    Brillouin-zone double convolution."""
    dims = (4, 6, 2, 4)
    N = 4
    S = oracle.smear(unit_links(dims), synth.point_source(dims, range(12)), dims, 0.25, N)
    L = dims[:3]
    Q = np.meshgrid(*[2 * np.pi * np.arange(l) / l for l in L], indexing="ij")
    lam = (1 + 0.5 * (np.cos(Q[0]) + np.cos(Q[1]) + np.cos(Q[2]))) ** N
    Vs = L[0] * L[1] * L[2]
    flat = lam.reshape(-1)
    idx = np.indices(L).reshape(3, -1)
    cube = 0.0
    for i in range(Vs):
        k = (idx[:, i:i + 1] + idx) % np.array(L)[:, None]
        cube += flat[i] * np.sum(flat * lam[k[0], k[1], k[2]])
    cube /= Vs ** 2
    for parity in (1, -1):
        G, Gp, P = _delta_gammas(parity)
        K = 0
        for g, gp in zip(G, Gp):
            K += (np.trace(g @ gp) * np.trace(P) + np.trace(g @ gp.T) * np.trace(P) + np.trace(g @ gp @ P.T)
                  + np.trace(g @ P @ gp) + np.trace(g @ P @ gp.T) + np.trace(g @ gp.T @ P.T))
        assert abs(K) > 1.0  # the pin is not trivially zero
        C = oracle.delta(S, dims, parity)
        assert abs(C[0] - 6 * K * cube) <= 1e-12 * abs(6 * K * cube)
        assert np.count_nonzero(C[1:]) == 0


def test_delta_gauge_invariance():
    dims = (4, 2, 2, 3)
    S = synth.gaussian_propagator(dims, 193)
    g = synth.gauge_transform(dims, 9193)
    C = oracle.delta(S, dims, 1)
    Cg = oracle.delta(gauge_rotate_fermions(g, S), dims, 1)
    assert np.abs(C - Cg).max() <= 1e-13 * np.abs(C).max()

    # a U(3) rotation exp(i theta(t)) g(x) at the sink multiplies C(t) by the
    # determinant exp(3 i theta(t)): exactly one epsilon tensor at the sink
    theta = np.array([0.3, -1.1, 2.0])
    Vs = 16
    ph = np.repeat(np.exp(1j * theta), Vs)[:, None, None] * g
    Cu = oracle.delta(gauge_rotate_fermions(ph, S), dims, 1)
    assert np.abs(Cu - np.exp(3j * theta) * C).max() <= 1e-13 * np.abs(C).max()


def test_config1_pion_is_column_norm_per_slice():
    """The one-column pion correlator C(t) = sum_x |psi(x, t)|^2 is the n = 15
    term restricted to column 0 (the other columns zero)."""
    dims = (4, 4, 4, 8)
    U = synth.su3_links(dims, 1)
    psi = oracle.smear(U, synth.point_source(dims, [0]), dims, 0.25, 10)
    S = np.zeros((12,) + psi.shape[1:], dtype=np.complex128)
    S[0] = psi[0]
    C = oracle.meson(S, S, dims)
    direct = np.sum(np.abs(psi[0]) ** 2, axis=(1, 2)).reshape(8, -1).sum(axis=1)
    assert np.abs(C[15] - direct).max() <= 1e-13 * direct.max()
    ts = oracle.timeslice_sum(np.sum(np.abs(psi[0]) ** 2, axis=(1, 2)), dims)[:, 0]
    assert np.abs(ts - direct).max() <= 1e-13 * direct.max()


# --------------------------------------------------------------------------
# Sums
# --------------------------------------------------------------------------

def test_sums_against_integer_fields():
    """Integer-valued fields make FP64 sums exact, independent of order."""
    dims = (4, 2, 2, 5)
    V = synth.volume(dims)
    rng = np.random.default_rng(3)
    f = rng.integers(-50, 50, size=(V, 3)) + 1j * rng.integers(-50, 50, size=(V, 3))
    ts = oracle.timeslice_sum(f, dims)
    assert np.array_equal(ts, f.reshape(5, -1, 3).sum(axis=1))
    assert oracle.norm2(f) == float(np.sum(np.abs(f) ** 2))
    g = rng.integers(-50, 50, size=(V, 3)) + 1j * rng.integers(-50, 50, size=(V, 3))
    assert oracle.inner(f, g) == complex(np.sum(np.conj(f) * g))


def test_golden_config1_regression():
    """Stored oracle output (tests/golden/make_golden.py) still reproduces."""
    import json
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "config1_fp64.json")
    gold = json.load(open(path))
    dims = (4, 4, 4, 8)
    psi = oracle.smear(synth.su3_links(dims, 1), synth.point_source(dims, [0]), dims, 0.25, 10)[0]
    corr = oracle.timeslice_sum(np.sum(np.abs(psi) ** 2, axis=(1, 2)), dims)[:, 0].real
    assert np.allclose(corr, gold["pion_correlator"], rtol=1e-13, atol=0)
    # locality: only the source slice is populated
    assert np.count_nonzero(corr[1:]) == 0
