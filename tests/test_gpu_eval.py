"""GPU parity: expression evaluation (qdp_eval, qdp_shift, qdp_sum_multi)
against the numpy expression oracle.  FP64 fields: 1e-12 relative; shifts
and copies are bitwise."""

import numpy as np
import pytest

import oracle
from oracle import expr as E
from paper_1111_5596_amd import synth

pytestmark = pytest.mark.gpu

DIMS = (4, 6, 2, 4)
V = synth.volume(DIMS)


def rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


SHAPES = {"REAL": (V,), "COMPLEX": (V,), "COLOR_VECTOR": (V, 3), "COLOR_MATRIX": (V, 3, 3),
          "FERMION": (V, 4, 3), "SPIN_MATRIX": (V, 4, 4), "PROPAGATOR": (V, 4, 4, 3, 3)}


@pytest.fixture(scope="module")
def env(qdp):
    lat = qdp.lattice(DIMS)
    host, handles = {}, {}
    specs = {"psi": "FERMION", "chi": "FERMION", "A": "COLOR_MATRIX", "B": "COLOR_MATRIX",
             "P": "PROPAGATOR", "Q": "PROPAGATOR", "M": "SPIN_MATRIX", "c": "COMPLEX",
             "r": "REAL", "v": "COLOR_VECTOR", "w": "COLOR_VECTOR"}
    for i, (k, t) in enumerate(specs.items()):
        a = rand(SHAPES[t], 100 + i)
        if t == "REAL":
            a = a.real
        h = qdp.alloc(lat, t, "F64")
        qdp.write(h, a)
        host[k] = (t, a)
        handles[k] = h
    U = synth.su3_links(DIMS, 8)
    g = qdp.alloc(lat, "GAUGE", "F64")
    qdp.write(g, U)
    host["U"] = ("GAUGE", U)
    handles["U"] = g
    yield qdp, lat, host, handles
    for h in handles.values():
        qdp.free(h)


def to_gpu(prog, handles):
    out = []
    for t in prog:
        if t[0] == "field":
            out.append(("field", handles[t[1]]))
        elif t[0] == "gauge":
            out.append(("gauge", handles[t[1]], t[2]))
        else:
            out.append(t)
    return out


PROGRAMS = [
    ("FERMION", [("field", "psi")]),
    ("FERMION", [("field", "psi"), ("shift", 2, -1)]),
    ("FERMION", [("field", "psi"), ("complex_const", 0.5, -1.5), ("mul",), ("field", "chi"), ("add",)]),
    ("FERMION", [("gauge", "U", 1), ("field", "psi"), ("shift", 1, 1), ("mul",)]),
    ("FERMION", [("gauge", "U", 0), ("adj",), ("field", "psi"), ("mul",), ("shift", 0, -1)]),
    ("FERMION", [("field", "M"), ("field", "psi"), ("mul",), ("gamma_left", 5), ("neg",)]),
    ("FERMION", [("field", "P"), ("field", "chi"), ("shift", 3, 1), ("mul",)]),
    ("FERMION", [("field", "psi"), ("field", "c"), ("mul",), ("field", "r"), ("field", "chi"), ("mul",), ("sub",)]),
    ("COLOR_MATRIX", [("field", "A"), ("field", "B"), ("adj",), ("mul",), ("shift", 2, 1)]),
    ("COLOR_MATRIX", [("field", "P"), ("trace_spin",), ("field", "A"), ("add",)]),
    ("COLOR_MATRIX", [("gauge", "U", 3), ("gauge", "U", 2), ("shift", 3, 1), ("mul",), ("conj",)]),
    ("SPIN_MATRIX", [("field", "P"), ("trace_color",), ("gamma_right", 11)]),
    ("PROPAGATOR", [("field", "P"), ("field", "Q"), ("mul",), ("gamma_left", 15)]),
    ("PROPAGATOR", [("field", "M"), ("field", "A"), ("mul",), ("field", "P"), ("adj",), ("add",)]),
    ("COMPLEX", [("field", "P"), ("field", "Q"), ("adj",), ("mul",), ("trace",)]),
    ("COMPLEX", [("field", "psi"), ("field", "chi"), ("local_inner",), ("field", "c"), ("conj",), ("mul",)]),
    ("REAL", [("field", "psi"), ("local_norm2",), ("field", "c"), ("imag",), ("add",)]),
    ("REAL", [("field", "c"), ("real",), ("field", "r"), ("shift", 1, -1), ("mul",)]),
    ("COLOR_VECTOR", [("field", "A"), ("field", "v"), ("mul",), ("field", "w"), ("shift", 0, 1), ("sub",)]),
    ("COMPLEX", [("field", "A"), ("trace",), ("real_const", 2.0), ("mul",)]),
    ("COMPLEX", [("field", "A"), ("field", "B"), ("shift", 0, 1), ("mul",), ("trace",)]),
    ("COMPLEX", [("field", "M"), ("field", "M"), ("gamma_left", 5), ("mul",), ("trace",)]),
]


@pytest.mark.parametrize("idx", range(len(PROGRAMS)))
@pytest.mark.parametrize("sub", ["all", "even", "odd", ("timeslice", 2)])
def test_eval_matches_oracle(env, idx, sub):
    q, lat, host, handles = env
    t, prog = PROGRAMS[idx]
    dest0 = rand(SHAPES[t], 999)
    if t == "REAL":
        dest0 = dest0.real
    d = q.alloc(lat, t, "F64")
    q.write(d, dest0)
    q.eval(to_gpu(prog, handles), d, sub)
    expect = E.assign(prog, host, DIMS, t, dest0, sub)
    got = q.read(d)
    assert np.abs(got - expect).max() <= 1e-12 * max(1.0, np.abs(expect).max())
    # sites outside the subset are untouched (bitwise)
    m = ~E.subset_mask(DIMS, sub)
    assert np.array_equal(got[m], np.asarray(dest0)[m])
    q.free(d)


@pytest.fixture(scope="module", params=["F32", "F16S"])
def env_low(qdp, request):
    """The same operands stored in FP32 or F16S; the oracle gets the stored
    (rounded) values read back."""
    prec = request.param
    lat = qdp.lattice(DIMS)
    host, handles = {}, {}
    specs = {"psi": "FERMION", "chi": "FERMION", "A": "COLOR_MATRIX", "B": "COLOR_MATRIX",
             "P": "PROPAGATOR", "Q": "PROPAGATOR", "M": "SPIN_MATRIX", "c": "COMPLEX",
             "r": "REAL", "v": "COLOR_VECTOR", "w": "COLOR_VECTOR"}
    for i, (k, t) in enumerate(specs.items()):
        a = rand(SHAPES[t], 100 + i)
        if t == "REAL":
            a = a.real
        h = qdp.alloc(lat, t, prec)
        qdp.write(h, a)
        host[k] = (t, qdp.read(h))
        handles[k] = h
    g = qdp.alloc(lat, "GAUGE", prec)
    qdp.write(g, synth.su3_links(DIMS, 8))
    host["U"] = ("GAUGE", qdp.read(g))
    handles["U"] = g
    yield qdp, lat, host, handles, prec
    for h in handles.values():
        qdp.free(h)


@pytest.mark.parametrize("idx", range(len(PROGRAMS)))
def test_eval_lower_precisions(env_low, idx):
    """Every program with all operands and the destination in FP32 or F16S
    storage (FP32 arithmetic): FP32 within 1e-5, F16S within 1e-3 of the
    largest result (one F16S rounding of the stored result is 2^-12 of its
    record's scale), on the full lattice and on the odd sites, whose
    complement keeps its stored values bitwise."""
    q, lat, host, handles, prec = env_low
    t, prog = PROGRAMS[idx]
    tol = {"F32": 1e-5, "F16S": 1e-3}[prec]
    for sub in ("all", "odd"):
        d = q.alloc(lat, t, prec)
        dest0 = rand(SHAPES[t], 999)
        q.write(d, dest0.real if t == "REAL" else dest0)
        dest0 = q.read(d)
        q.eval(to_gpu(prog, handles), d, sub)
        expect = E.assign(prog, host, DIMS, t, dest0, sub)
        got = q.read(d)
        assert np.abs(got - expect).max() <= tol * max(1.0, np.abs(expect).max()), (prec, sub)
        m = ~E.subset_mask(DIMS, sub)
        assert np.array_equal(got[m], np.asarray(dest0)[m])
        q.free(d)


@pytest.mark.parametrize("op", ["+=", "-=", "*="])
def test_compound_assign(env, op):
    q, lat, host, handles = env
    d = q.alloc(lat, "COLOR_MATRIX", "F64")
    start = rand((V, 3, 3), 77)
    q.write(d, start)
    prog = [("field", "A"), ("gauge", "U", 1), ("mul",)]
    q.eval(to_gpu(prog, handles), d, "all", op)
    expect = E.assign(prog, host, DIMS, "COLOR_MATRIX", start, "all", op)
    assert np.abs(q.read(d) - expect).max() <= 1e-12 * np.abs(expect).max()
    q.free(d)


def test_shift_bitwise_and_round_trip(env):
    q, lat, host, handles = env
    a = q.alloc(lat, "PROPAGATOR", "F64")
    b = q.alloc(lat, "PROPAGATOR", "F64")
    P = host["P"][1]
    for mu in range(4):
        for sign in (1, -1):
            q.shift(a, handles["P"], mu, sign)
            assert np.array_equal(q.read(a), oracle.shift(P, DIMS, mu, sign))
            q.shift(b, a, mu, -sign)
            assert np.array_equal(q.read(b), P)
    q.free(a)
    q.free(b)


def test_alias_and_type_errors(env):
    from paper_1111_5596_amd.qdpmi import QdpError

    q, lat, host, handles = env
    with pytest.raises(QdpError, match="ALIAS"):
        q.shift(handles["psi"], handles["psi"], 0, 1)
    with pytest.raises(QdpError, match="ALIAS"):
        q.eval([("field", handles["psi"]), ("field", handles["psi"]), ("shift", 1, 1), ("add",)],
               handles["psi"])
    with pytest.raises(QdpError, match="TYPE"):
        q.eval([("field", handles["psi"]), ("field", handles["psi"]), ("mul",)], handles["chi"])
    with pytest.raises(QdpError, match="TYPE"):
        q.eval([("field", handles["A"])], handles["psi"])
    other = q.alloc(q.lattice((4, 4, 4, 4)), "FERMION", "F64")
    with pytest.raises(QdpError, match="LATTICE"):
        q.eval([("field", other)], handles["psi"])
    q.free(other)
    # in-place unshifted update is allowed: psi = 2 psi
    d = q.alloc(lat, "FERMION", "F64")
    q.write(d, host["psi"][1])
    q.eval([("field", d), ("real_const", 2.0), ("mul",)], d)
    assert np.array_equal(q.read(d), 2 * host["psi"][1])
    q.free(d)


@pytest.mark.parametrize("kind,nsub", [("all", 1), ("parity", 2), ("timeslice", DIMS[3])])
def test_sum_multi(env, kind, nsub):
    q, lat, host, handles = env
    # the first six are formed inside the reduction (local norm, inner
    # product, trace, trace of a product; shifted, and an evaluated operand),
    # the others reduce a field or an evaluated temporary component-wise
    for t, prog in [("REAL", [("field", "psi"), ("local_norm2",)]),
                    ("COMPLEX", [("field", "P"), ("field", "Q"), ("mul",), ("trace",)]),
                    ("COMPLEX", [("field", "psi"), ("field", "chi"), ("shift", 1, -1), ("local_inner",)]),
                    ("COMPLEX", [("field", "A"), ("shift", 3, 1), ("trace",)]),
                    ("REAL", [("field", "psi"), ("field", "chi"), ("sub",), ("local_norm2",)]),
                    ("COMPLEX", [("field", "A"), ("field", "B"), ("adj",), ("mul",), ("trace",)]),
                    ("COLOR_MATRIX", [("field", "A")]),
                    ("PROPAGATOR", [("field", "P")]),
                    ("SPIN_MATRIX", [("field", "P"), ("trace_color",)]),
                    ("FERMION", [("gauge", "U", 2), ("field", "psi"), ("shift", 2, 1), ("mul",)])]:
        ncomp = {"REAL": 1, "COMPLEX": 1, "COLOR_MATRIX": 9, "FERMION": 12, "PROPAGATOR": 144,
                 "SPIN_MATRIX": 16}[t]
        got = q.sum_multi(to_gpu(prog, handles), kind, ncomp, nsub)
        _, expect = E.sum_multi(prog, host, DIMS, kind)
        assert np.abs(got - expect).max() <= 1e-12 * np.abs(expect).max()
        got2 = q.sum_multi(to_gpu(prog, handles), kind, ncomp, nsub)
        assert np.array_equal(got, got2)


@pytest.mark.parametrize("prec", ["F32", "F16S"])
def test_local_reductions_of_stored_fields(qdp, prec):
    """|psi|^2 and psi^dagger chi formed inside the reduction from FP32 and
    F16S fields, every slice: FP64 sums of the decoded stored values."""
    dims = (6, 4, 4, 6)
    lat = qdp.lattice(dims)
    psi, chi = synth.gaussian_propagator(dims, 131, ncols=2)
    a, b = qdp.alloc(lat, "FERMION", prec), qdp.alloc(lat, "FERMION", prec)
    qdp.write(a, psi)
    qdp.write(b, chi)
    pa, pb = qdp.read(a), qdp.read(b)
    vs = dims[0] * dims[1] * dims[2]
    n2 = qdp.sum_multi([("field", a), ("local_norm2",)], "timeslice", 1, dims[3])[:, 0]
    ip = qdp.sum_multi([("field", a), ("field", b), ("local_inner",)], "timeslice", 1, dims[3])[:, 0]
    for t in range(dims[3]):
        sl = slice(t * vs, (t + 1) * vs)
        e_n2 = np.sum(np.abs(pa[sl]) ** 2)
        e_ip = np.sum(np.conj(pa[sl]) * pb[sl])
        assert abs(n2[t] - e_n2) <= 1e-13 * e_n2 and n2[t].imag == 0
        assert abs(ip[t] - e_ip) <= 1e-13 * e_n2
    qdp.free(a)
    qdp.free(b)


@pytest.mark.parametrize("prec", ["F32", "F64", "F16S"])
def test_jacobi_expression_stencil(qdp, prec):
    """The whole Jacobi step written as one expression (fused stencil path)."""
    dims = (8, 4, 6, 2)
    U = synth.su3_links(dims, 12)
    psi = synth.gaussian_propagator(dims, 112, ncols=1)[0]
    lat = qdp.lattice(dims)
    g = qdp.alloc(lat, "GAUGE", prec)
    qdp.write(g, U)
    a = qdp.alloc(lat, "FERMION", prec)
    qdp.write(a, psi)
    b = qdp.alloc(lat, "FERMION", prec)
    prog = [("field", a)]
    for i in range(3):
        prog += [("gauge", g, i), ("field", a), ("shift", i, 1), ("mul",), ("real_const", 0.25), ("mul",), ("add",)]
        prog += [("gauge", g, i), ("adj",), ("field", a), ("mul",), ("shift", i, -1), ("real_const", 0.25),
                 ("mul",), ("add",)]
    qdp.eval(prog, b)
    ref_in = qdp.read(a)
    Ur = qdp.read(g)
    expect = oracle.smear_step(Ur, ref_in, dims, 0.25)
    tol = {"F64": 1e-13, "F32": 1e-6, "F16S": 1e-3}[prec]
    got = qdp.read(b)
    assert np.linalg.norm(got - expect) <= tol * np.linalg.norm(expect)
    for f in (g, a, b):
        qdp.free(f)


@pytest.mark.parametrize("ftype,prec", [("FERMION", "F32"), ("GAUGE", "F16S"), ("REAL", "F64"),
                                        ("PROPAGATOR", "F64")])
def test_read_timeslices_matches_full_read(qdp, ftype, prec):
    dims = (6, 4, 2, 10)
    lat = qdp.lattice(dims)
    f = qdp.alloc(lat, ftype, prec)
    V = synth.volume(dims)
    shape = {"FERMION": (V, 4, 3), "GAUGE": (4, V, 3, 3), "REAL": (V,), "PROPAGATOR": (V, 4, 4, 3, 3)}[ftype]
    a = rand(shape, 5)
    qdp.write(f, a.real if ftype == "REAL" else a)
    full = qdp.read(f)
    Vs = 6 * 4 * 2
    for t0, t1 in [(0, 1), (3, 7), (9, 10), (0, 10)]:
        part = qdp.read_timeslices(f, t0, t1)
        if ftype == "GAUGE":
            assert np.array_equal(part, full[:, t0 * Vs:t1 * Vs])
        else:
            assert np.array_equal(part, full[t0 * Vs:t1 * Vs])
    qdp.free(f)
