"""Pins of the numpy expression oracle (QDP-style site-local expressions).

The expression oracle is checked against the C oracle (an independent
implementation of the smearing step and of shift), against algebraic
identities (adjoint, trace cyclicity, partial traces, gamma squares) and
against its own type rules."""

import numpy as np
import pytest

import oracle
from oracle import expr as E
from paper_1111_5596_amd import synth


def rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


DIMS = (4, 2, 6, 4)
V = synth.volume(DIMS)


def fields():
    U = synth.su3_links(DIMS, 3)
    return {
        "U": ("GAUGE", U),
        "psi": ("FERMION", rand((V, 4, 3), 1)),
        "chi": ("FERMION", rand((V, 4, 3), 2)),
        "A": ("COLOR_MATRIX", rand((V, 3, 3), 3)),
        "B": ("COLOR_MATRIX", rand((V, 3, 3), 4)),
        "P": ("PROPAGATOR", rand((V, 4, 4, 3, 3), 5)),
        "Q": ("PROPAGATOR", rand((V, 4, 4, 3, 3), 6)),
        "M": ("SPIN_MATRIX", rand((V, 4, 4), 7)),
        "c": ("COMPLEX", rand((V,), 8)),
        "r": ("REAL", rand((V,), 9).real),
        "v": ("COLOR_VECTOR", rand((V, 3), 10)),
    }


def ev(prog, f=None):
    t, a = E.evaluate(prog, fields() if f is None else f, DIMS)
    return t, E.to_canonical(t, a)


def jacobi_program(kappa):
    """psi + kappa * sum_i [U_i psi(x+i) + shift(adj(U_i) psi, -i)]"""
    prog = [("field", "psi")]
    for i in range(3):
        prog += [("gauge", "U", i), ("field", "psi"), ("shift", i, +1), ("mul",),
                 ("real_const", kappa), ("mul",), ("add",)]
        prog += [("gauge", "U", i), ("adj",), ("field", "psi"), ("mul",), ("shift", i, -1),
                 ("real_const", kappa), ("mul",), ("add",)]
    return prog


def test_jacobi_expression_matches_c_smear_step():
    f = fields()
    t, got = ev(jacobi_program(0.25), f)
    assert t == "FERMION"
    expect = oracle.smear_step(f["U"][1], f["psi"][1], DIMS, 0.25)
    assert np.abs(got - expect).max() <= 1e-14 * np.abs(expect).max()


def test_shift_matches_c_shift():
    f = fields()
    for mu in range(4):
        for sign in (+1, -1):
            _, got = ev([("field", "P"), ("shift", mu, sign)], f)
            assert np.array_equal(got, oracle.shift(f["P"][1], DIMS, mu, sign))


def test_adjoint_identities():
    f = fields()
    _, a = ev([("field", "A"), ("adj",), ("adj",)], f)
    assert np.array_equal(a, f["A"][1])
    _, lhs = ev([("field", "A"), ("field", "B"), ("mul",), ("adj",)], f)
    _, rhs = ev([("field", "B"), ("adj",), ("field", "A"), ("adj",), ("mul",)], f)
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-13)
    _, lhs = ev([("field", "P"), ("field", "Q"), ("mul",), ("adj",)], f)
    _, rhs = ev([("field", "Q"), ("adj",), ("field", "P"), ("adj",), ("mul",)], f)
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-12)
    # SU(3): U^dagger U = 1
    _, uu = ev([("gauge", "U", 2), ("adj",), ("gauge", "U", 2), ("mul",)], f)
    assert np.abs(uu - np.eye(3)).max() < 1e-14


def test_trace_identities():
    f = fields()
    _, t1 = ev([("field", "P"), ("field", "Q"), ("mul",), ("trace",)], f)
    _, t2 = ev([("field", "Q"), ("field", "P"), ("mul",), ("trace",)], f)
    assert np.allclose(t1, t2, rtol=0, atol=1e-12)
    _, full = ev([("field", "P"), ("trace",)], f)
    _, cs = ev([("field", "P"), ("trace_color",), ("trace",)], f)
    _, sc = ev([("field", "P"), ("trace_spin",), ("trace",)], f)
    assert np.allclose(full, cs, atol=1e-13) and np.allclose(full, sc, atol=1e-13)
    t, tc = ev([("field", "P"), ("trace_color",)], f)
    assert t == "SPIN_MATRIX" and tc.shape == (V, 4, 4)
    t, ts = ev([("field", "P"), ("trace_spin",)], f)
    assert t == "COLOR_MATRIX" and ts.shape == (V, 3, 3)
    # explicit index sums
    P = f["P"][1]
    assert np.allclose(tc, np.einsum("vijaa->vij", P)) and np.allclose(ts, np.einsum("viiab->vab", P))


def test_product_type_rules():
    cases = {
        ("A", "v"): "COLOR_VECTOR", ("A", "psi"): "FERMION", ("M", "psi"): "FERMION",
        ("M", "A"): "PROPAGATOR", ("A", "M"): "PROPAGATOR", ("P", "psi"): "FERMION",
        ("P", "A"): "PROPAGATOR", ("c", "psi"): "FERMION", ("psi", "r"): "FERMION",
        ("r", "r"): "REAL", ("r", "c"): "COMPLEX", ("M", "M"): "SPIN_MATRIX",
    }
    for (a, b), t in cases.items():
        assert ev([("field", a), ("field", b), ("mul",)])[0] == t
    for a, b in [("psi", "psi"), ("v", "A"), ("psi", "A"), ("v", "M"), ("psi", "P")]:
        with pytest.raises(E.ExprTypeError):
            ev([("field", a), ("field", b), ("mul",)])
    for prog in ([("field", "psi"), ("adj",)], [("field", "v"), ("trace",)],
                 [("field", "A"), ("gamma_left", 3)], [("field", "psi"), ("gamma_right", 1)],
                 [("field", "psi"), ("field", "A"), ("add",)], [("field", "A"), ("real",)]):
        with pytest.raises(E.ExprTypeError):
            ev(prog)


def test_product_matches_explicit_sums():
    f = fields()
    A, psi, M, P = f["A"][1], f["psi"][1], f["M"][1], f["P"][1]
    _, got = ev([("field", "A"), ("field", "psi"), ("mul",)], f)
    assert np.allclose(got, np.einsum("vab,vsb->vsa", A, psi), atol=1e-13)
    _, got = ev([("field", "M"), ("field", "psi"), ("mul",)], f)
    assert np.allclose(got, np.einsum("vst,vta->vsa", M, psi), atol=1e-13)
    _, got = ev([("field", "P"), ("field", "psi"), ("mul",)], f)
    assert np.allclose(got, np.einsum("vstab,vtb->vsa", P, psi), atol=1e-12)
    _, got = ev([("field", "M"), ("field", "A"), ("mul",)], f)
    assert np.allclose(got, np.einsum("vst,vab->vstab", M, A), atol=1e-13)


def test_gamma_products():
    f = fields()
    for n in range(16):
        k = bin(n).count("1")
        eps = (-1) ** (k * (k - 1) // 2)
        _, got = ev([("field", "psi"), ("gamma_left", n), ("gamma_left", n)], f)
        assert np.allclose(got, eps * f["psi"][1], atol=1e-14)


# DeGrand-Rossi gamma_1..gamma_4 written out as dense matrices, independent of
# the oracle's tables; Gamma_n = gamma_1^b0 gamma_2^b1 gamma_3^b2 gamma_4^b3
# for the bits b_k of n.
_DR = [np.array(m, dtype=np.complex128) for m in (
    [[0, 0, 0, 1j], [0, 0, 1j, 0], [0, -1j, 0, 0], [-1j, 0, 0, 0]],
    [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],
    [[0, 0, 1j, 0], [0, 0, 0, -1j], [-1j, 0, 0, 0], [0, 1j, 0, 0]],
    [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]])]


def _gamma_written_out(n):
    g = np.eye(4, dtype=np.complex128)
    for k in range(4):
        if (n >> k) & 1:
            g = g @ _DR[k]
    return g


def _basis_fields(dims):
    """Every spin basis element at its own site: SPIN_MATRIX E_{ij} at site
    4 i + j and FERMION e_{s,a} (spin s, colour a) at site 3 s + a; zero
    elsewhere.  Applying a 4x4 matrix G to them reads G off entry by entry."""
    V = synth.volume(dims)
    assert V >= 16
    M = np.zeros((V, 4, 4), dtype=np.complex128)
    psi = np.zeros((V, 4, 3), dtype=np.complex128)
    for i in range(4):
        for j in range(4):
            M[4 * i + j, i, j] = 1.0
    for s in range(4):
        for a in range(3):
            psi[3 * s + a, s, a] = 1.0
    return M, psi


@pytest.mark.parametrize("n", range(16))
def test_gamma_left_right_match_written_out_products(n):
    """gamma_left(n) a = Gamma_n a and gamma_right(n) a = a Gamma_n on basis
    fields, Gamma_n built here from the written-out gamma_1..gamma_4 in the
    order gamma_1^b0 gamma_2^b1 gamma_3^b2 gamma_4^b3.  The transpose, the
    adjoint or the reversed product of Gamma_n fails for some n (checked
    below), so each entry of the operation is pinned."""
    G = _gamma_written_out(n)
    M, psi = _basis_fields(DIMS)
    f = {"M": ("SPIN_MATRIX", M), "psi": ("FERMION", psi)}
    _, gl = ev([("field", "M"), ("gamma_left", n)], f)
    _, gr = ev([("field", "M"), ("gamma_right", n)], f)
    _, gp = ev([("field", "psi"), ("gamma_left", n)], f)
    for i in range(4):
        for j in range(4):
            E_ij = np.zeros((4, 4))
            E_ij[i, j] = 1.0
            assert np.array_equal(gl[4 * i + j], G @ E_ij)
            assert np.array_equal(gr[4 * i + j], E_ij @ G)
    for s in range(4):
        for a in range(3):
            # Gamma e_{s,a}: column s of Gamma in colour a
            expect = np.zeros((4, 3), dtype=np.complex128)
            expect[:, a] = G[:, s]
            assert np.array_equal(gp[3 * s + a], expect)
    assert not np.any(gl[16:]) and not np.any(gp[12:])


def test_gamma_written_out_products_discriminate():
    """The pins above would catch the plausible mistakes: for some n the
    transpose, the adjoint and the reversed-order product all differ from
    Gamma_n."""
    def reversed_product(n):
        g = np.eye(4, dtype=np.complex128)
        for k in reversed(range(4)):
            if (n >> k) & 1:
                g = g @ _DR[k]
        return g

    G = [_gamma_written_out(n) for n in range(16)]
    assert any(not np.allclose(g, g.T) for g in G)
    assert any(not np.allclose(g, g.conj().T) for g in G)
    assert any(not np.allclose(G[n], reversed_product(n)) for n in range(16))
    # gamma_5 = Gamma_15 = diag(1, 1, -1, -1) in this basis
    assert np.allclose(G[15], np.diag([1, 1, -1, -1]))


def _propagator_from_columns(S):
    """12 FERMION columns (12, V, 4, 3) -> PROPAGATOR (V, 4, 4, 3, 3) with
    P[x, s, s', a, a'] = component (s, a) of column 3 s' + a'."""
    V = S.shape[1]
    return np.transpose(S.reshape(4, 3, V, 4, 3), (2, 3, 0, 4, 1))


def test_meson_from_expression_programs_matches_contraction():
    """C_n(t) = sum_{x in t} Tr[gamma_5 S2^dagger gamma_5 Gamma_n S1 Gamma_n]
    written as an expression program (gamma_left / gamma_right, adj, product,
    trace, time-slice sum) equals the C oracle's contraction on a 2^4 lattice
    for every n: the expression operations and the contraction are two
    independent codings of the same formula."""
    dims = (2, 2, 2, 2)
    S1 = synth.gaussian_propagator(dims, 211)
    S2 = synth.gaussian_propagator(dims, 212)
    f = {"S1": ("PROPAGATOR", _propagator_from_columns(S1)),
         "S2": ("PROPAGATOR", _propagator_from_columns(S2))}
    ref = oracle.meson(S1, S2, dims)
    for n in range(16):
        prog = [("field", "S2"), ("adj",), ("gamma_left", 15), ("gamma_right", 15),
                ("field", "S1"), ("gamma_left", n), ("gamma_right", n), ("mul",), ("trace",)]
        _, got = E.sum_multi(prog, f, dims, "timeslice")
        assert np.abs(got[:, 0] - ref[n]).max() <= 1e-13 * np.abs(ref[15]).max(), n
def test_local_norm_and_inner():
    f = fields()
    t, n2 = ev([("field", "psi"), ("local_norm2",)], f)
    assert t == "REAL"
    t, ii = ev([("field", "psi"), ("field", "psi"), ("local_inner",)], f)
    assert t == "COMPLEX"
    assert np.allclose(n2, ii.real, atol=1e-13) and np.abs(ii.imag).max() < 1e-13
    t, re = ev([("field", "c"), ("real",)], f)
    _, im = ev([("field", "c"), ("imag",)], f)
    assert t == "REAL" and np.array_equal(re + 1j * im, f["c"][1])


def test_subsets_partition_and_assign_ops():
    f = fields()
    dest = np.zeros((V, 4, 3), dtype=complex)
    prog = [("field", "psi"), ("complex_const", 0.5, -2.0), ("mul",)]
    even = E.assign(prog, f, DIMS, "FERMION", dest, "even")
    both = E.assign(prog, f, DIMS, "FERMION", even, "odd")
    full = E.assign(prog, f, DIMS, "FERMION", dest, "all")
    assert np.array_equal(both, full)
    m = E.subset_mask(DIMS, "even")
    assert np.count_nonzero(even[~m]) == 0 and m.sum() == V // 2
    pieces = dest
    for t in range(DIMS[3]):
        pieces = E.assign(prog, f, DIMS, "FERMION", pieces, ("timeslice", t))
    assert np.array_equal(pieces, full)
    add = E.assign([("field", "chi")], f, DIMS, "FERMION", full, "all", "+=")
    assert np.allclose(add, full + f["chi"][1])
    mul = E.assign([("field", "A")], f, DIMS, "COLOR_MATRIX", f["B"][1], "all", "*=")
    assert np.allclose(mul, np.einsum("vab,vbc->vac", f["B"][1], f["A"][1]))
    with pytest.raises(E.ExprTypeError):
        E.assign([("field", "A")], f, DIMS, "FERMION", dest)


def test_sum_multi_matches_c_sums():
    f = fields()
    t, s = E.sum_multi([("field", "psi"), ("local_norm2",)], f, DIMS, "timeslice")
    per_site = np.sum(np.abs(f["psi"][1]) ** 2, axis=(1, 2))
    expect = oracle.timeslice_sum(per_site, DIMS)
    assert np.allclose(s, expect, rtol=1e-14)
    t, s = E.sum_multi([("field", "psi"), ("field", "chi"), ("local_inner",)], f, DIMS, "all")
    assert abs(s[0, 0] - oracle.inner(f["psi"][1], f["chi"][1])) < 1e-11
    t, s = E.sum_multi([("field", "A")], f, DIMS, "parity")
    m = E.subset_mask(DIMS, "even")
    assert np.allclose(s[0], f["A"][1][m].reshape(-1, 9).sum(axis=0))
