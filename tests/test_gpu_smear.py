"""GPU parity: Jacobi smearing through the C ABI against the FP64 oracle.

Tolerances (relative L2 over the whole field, a reference zero must stay an
exact zero): FP64 1e-12, FP32 1e-5, F16S 2e-3.  Free-field cases with
kappa = 1/4 are exact rationals and must match bitwise (FP64 for N <= 15,
FP32 for N <= 7).  Launch shapes, even/odd passes, graph replay and the
multi-lattice kernel must agree bitwise with each other."""

import numpy as np
import pytest

import oracle
from paper_1111_5596_amd import synth

pytestmark = pytest.mark.gpu

TOL = {"F64": 1e-12, "F32": 1e-5, "F16S": 2e-3}


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def upload(q, dims, U, cols, prec):
    lat = q.lattice(dims)
    g = q.alloc(lat, "GAUGE", prec)
    q.write(g, U)
    fs = []
    for c in cols:
        f = q.alloc(lat, "FERMION", prec)
        q.write(f, c)
        fs.append(f)
    return lat, g, fs


def free_all(q, fields):
    for f in fields:
        q.free(f)


def unit_links(dims):
    U = np.zeros((4, synth.volume(dims), 3, 3), dtype=np.complex128)
    U[:] = np.eye(3)
    return U


@pytest.mark.parametrize("prec", ["F64", "F32"])
def test_plain_method_4cubed(qdp, prec):
    """4^3 x 8, Haar links seed 1, point source column 0, kappa 0.25, N 10."""
    dims = (4, 4, 4, 8)
    U = synth.su3_links(dims, 1)
    src = synth.point_source(dims, [0])
    expect = oracle.smear(U, src, dims, 0.25, 10)[0]
    lat, g, (f,) = upload(qdp, dims, U, src, prec)
    qdp.smear(g, [f], 0.25, 10)
    got = qdp.read(f)
    assert rel(got, expect) <= TOL[prec]
    # pion correlator C(t) = sum_x |psi(x, t)|^2 via the FP64 time-slice sums
    corr = qdp.sum_multi([("field", f), ("local_norm2",)], "timeslice", 1, dims[3])[:, 0].real
    ref = oracle.timeslice_sum(np.sum(np.abs(expect) ** 2, axis=(1, 2)), dims)[:, 0].real
    assert np.count_nonzero(corr[1:]) == 0
    assert abs(corr[0] - ref[0]) <= TOL[prec] * ref[0]
    free_all(qdp, [g, f])


@pytest.mark.parametrize("prec,n", [("F64", 10), ("F64", 15), ("F32", 7)])
def test_free_field_bitwise(qdp, prec, n):
    dims = (4, 4, 4, 8)
    U = unit_links(dims)
    src = synth.point_source(dims, [0, 5])
    expect = oracle.smear(U, src, dims, 0.25, n)
    lat, g, fs = upload(qdp, dims, U, src, prec)
    qdp.smear(g, fs, 0.25, n, mode=1)
    for c in range(2):
        assert np.array_equal(qdp.read(fs[c]), expect[c])
    free_all(qdp, [g] + fs)


@pytest.mark.parametrize("prec", ["F64", "F32", "F16S"])
@pytest.mark.parametrize("dims,ncols,n", [((8, 8, 8, 4), 12, 9), ((6, 4, 10, 2), 5, 6),
                                          ((2, 2, 2, 2), 12, 10)])
def test_random_links_multi_column(qdp, prec, dims, ncols, n):
    U = synth.su3_links(dims, 7)
    psi = synth.gaussian_propagator(dims, 107, ncols=ncols)
    expect = oracle.smear(U, psi, dims, 0.25, n)
    lat, g, fs = upload(qdp, dims, U, psi, prec)
    qdp.smear(g, fs, 0.25, n)
    for c in range(ncols):
        assert rel(qdp.read(fs[c]), expect[c]) <= TOL[prec], (prec, c)
    free_all(qdp, [g] + fs)


@pytest.mark.parametrize("prec", ["F32", "F16S"])
def test_even_odd_equals_full_bitwise(qdp, prec):
    dims = (8, 4, 6, 4)
    U = synth.su3_links(dims, 3)
    psi = synth.gaussian_propagator(dims, 103, ncols=12)
    lat, g, a = upload(qdp, dims, U, psi, prec)
    b = []
    for c in psi:
        f = qdp.alloc(lat, "FERMION", prec)
        qdp.write(f, c)
        b.append(f)
    qdp.smear(g, a, 0.25, 7, mode=0)
    qdp.smear(g, b, 0.25, 7, mode=1)
    for x, y in zip(a, b):
        assert np.array_equal(qdp.read(x), qdp.read(y))
    free_all(qdp, [g] + a + b)


@pytest.mark.parametrize("prec", ["F64", "F32", "F16S"])
def test_launch_shapes_bitwise(qdp, prec):
    dims = (8, 8, 4, 4)
    U = synth.su3_links(dims, 4)
    psi = synth.gaussian_propagator(dims, 104, ncols=12)
    lat, g, fs = upload(qdp, dims, U, psi, prec)
    out = qdp.alloc(lat, "FERMION", prec)
    ref = None
    try:
        for shape in [(1, 1, 0, 0, 0, 0), (4, 1, 1, 2, 0, 0), (2, 2, 1, 3, 0, 0), (1, 3, 0, 2, 1, 0),
                      (1, 4, 1, 0, 1, 0), (2, 1, 0, 3, 1, 0), (4, 1, 1, 2, 1, 0), (2, 1, 1, 2, 0, 1),
                      (4, 1, 0, 0, 1, 1), (2, 2, 1, 3, 0, 1), (4, 1, 2, 0, 0, 1), (2, 2, 2, 2, 1, 1)]:
            qdp.set_shape(*shape)
            outs = [qdp.alloc(lat, "FERMION", prec) for _ in fs]
            qdp.smear_to(g, fs, outs, 0.25, 5, mode=1)
            assert qdp.get_shape()[:6] == shape
            vals = [qdp.read(o) for o in outs]
            if ref is None:
                ref = vals
            for v, r in zip(vals, ref):
                assert np.array_equal(v, r), shape
            free_all(qdp, outs)
    finally:
        qdp.set_shape(0)
    # inputs untouched by the out-of-place call
    for f, c in zip(fs, psi):
        if prec == "F32":
            assert np.array_equal(qdp.read(f), c.astype(np.complex64).astype(np.complex128))
    free_all(qdp, [g, out] + fs)


@pytest.mark.parametrize("dims", [(8, 8, 4, 4), (12, 12, 12, 4), (20, 20, 4, 2), (24, 12, 4, 2), (6, 6, 2, 2),
                                  (48, 48, 8, 4), (16, 2, 4, 2), (16, 32, 4, 2), (64, 4, 4, 2), (68, 4, 2, 2)])
@pytest.mark.parametrize("source", ["gaussian", "point"])
def test_lds_window_kernel_bitwise(qdp, dims, source):
    """The whole-lattice F16S kernel that stages the x/y neighbour window in
    LDS (blocks of 2 S waves over 64 S indices of both parities), S = 1, 2,
    both block mappings, plain order and two, three or four y bands
    (zstack 1, 2; bands apply where a band of a plane is whole blocks: 48^2
    planes with two bands for S = 1 and three for S = 2, 16 x 32 planes with
    every S and band count),
    against the kernels without LDS in both modes: windows that cover the
    whole parity range, a block range past the end of a parity (12^3 x 4:
    3456 indices per parity), y hops that wrap out of the window (20^2 and
    48^2 planes) and Ly = 2, the widest window (Lx = 64: the window is then
    exactly the LDS rows, 64 (S + 1) indices) and a lattice too wide for it
    (Lx = 68: the LDS shapes run the kernel without LDS); point sources
    (all-zero records beside non-zero ones) and Gaussian columns."""
    U = synth.su3_links(dims, 17)
    if source == "point":
        psi = synth.point_source(dims, range(12), site=synth.volume(dims) // 3)
    else:
        psi = synth.gaussian_propagator(dims, 117, ncols=12)
    lat, g, fs = upload(qdp, dims, U, psi, "F16S")
    try:
        ref = None
        for shape, mode in [((1, 1, 0, 0, 0, 0, 0), 1), ((4, 1, 1, 2, 0, 1, 0), 0), ((1, 1, 0, 0, 0, 0, 1), 0),
                            ((1, 1, 1, 0, 0, 0, 1), 0), ((1, 1, 0, 0, 0, 0, 2), 0), ((1, 1, 1, 0, 0, 0, 2), 0),
                            ((1, 1, 1, 0, 0, 1, 1), 0), ((1, 1, 0, 0, 0, 1, 1), 0), ((1, 1, 1, 0, 0, 2, 1), 0),
                            ((1, 1, 1, 0, 0, 1, 2), 0), ((1, 1, 1, 0, 0, 2, 2), 0)]:
            qdp.set_shape(*shape)
            outs = [qdp.alloc(lat, "FERMION", "F16S") for _ in fs]
            qdp.smear_to(g, fs, outs, 0.25, 6, mode=mode)
            assert qdp.get_shape() == shape
            vals = [qdp.read(o) for o in outs]
            if ref is None:
                ref = vals
                ex = oracle.smear(U, psi[[0, 5]], dims, 0.25, 6)
                for k, c in enumerate((0, 5)):
                    assert rel(vals[c], ex[k]) <= 2e-3, (dims, source, c)
            for v, r in zip(vals, ref):
                assert np.array_equal(v, r), (shape, mode)
            free_all(qdp, outs)
    finally:
        qdp.set_shape(0)
    free_all(qdp, [g] + fs)


@pytest.mark.parametrize("dims", [(16, 16, 4, 4), (24, 12, 4, 2), (20, 20, 4, 2), (6, 6, 2, 2)])
def test_zstacked_blocks_bitwise(qdp, dims):
    """Blocks whose wavefronts take tiles one (x, y) plane apart, against
    consecutive tiles, both modes: one parity's planes of 128, 144, 200 and
    18 sites (tile strides 2, 2, 3 and 1) and tile groups that run past the
    end of a parity (18 tiles per parity in groups of 8, 25 in groups of 12);
    zstack = 2 puts both parities' tiles in one block on the whole lattice."""
    U = synth.su3_links(dims, 16)
    psi = synth.gaussian_propagator(dims, 116, ncols=12)
    lat, g, fs = upload(qdp, dims, U, psi, "F32")
    try:
        for mode in (0, 1):
            ref = None
            for shape in [(1, 1, 0, 0, 0, 0), (2, 1, 0, 2, 0, 1), (4, 1, 1, 0, 0, 1), (2, 2, 1, 3, 1, 1),
                          (4, 1, 2, 2, 0, 1), (2, 1, 2, 0, 1, 1), (4, 1, 2, 2, 0, 2), (2, 1, 0, 0, 0, 2),
                          (4, 1, 1, 2, 1, 2)]:
                qdp.set_shape(*shape)
                outs = [qdp.alloc(lat, "FERMION", "F32") for _ in fs]
                qdp.smear_to(g, fs, outs, 0.25, 3, mode=mode)
                vals = [qdp.read(o) for o in outs]
                if ref is None:
                    ref = vals
                for v, r in zip(vals, ref):
                    assert np.array_equal(v, r), (shape, mode)
                free_all(qdp, outs)
    finally:
        qdp.set_shape(0)
    free_all(qdp, [g] + fs)


def test_graph_replay_equals_eager(qdp):
    from paper_1111_5596_amd import qdpmi

    dims = (8, 4, 4, 4)
    U = synth.su3_links(dims, 5)
    psi = synth.gaussian_propagator(dims, 105, ncols=3)
    eager = qdpmi.Context(pool_bytes=1 << 30, flags=qdpmi.INIT_NO_GRAPH | qdpmi.INIT_NO_AUTOTUNE)
    try:
        res = []
        for q in (qdp, eager):
            lat, g, fs = upload(q, dims, U, psi, "F32")
            for rep in range(3):  # replays of the cached graph
                q.smear(g, fs, 0.25, 4)
            res.append([q.read(f) for f in fs])
            free_all(q, [g] + fs)
        for a, b in zip(*res):
            assert np.array_equal(a, b)
    finally:
        eager.close()


def test_graph_cache_eviction(qdp):
    """More distinct smearing calls than the graph cache holds (16): the least
    recently used graphs are destroyed and rebuilt when needed again, and every
    result equals the eager launches' bitwise."""
    from paper_1111_5596_amd import qdpmi

    dims = (4, 4, 2, 2)
    U = synth.su3_links(dims, 6)
    psi = synth.gaussian_propagator(dims, 106, ncols=20)
    eager = qdpmi.Context(pool_bytes=1 << 28, flags=qdpmi.INIT_NO_GRAPH | qdpmi.INIT_NO_AUTOTUNE)
    try:
        res = []
        for q in (qdp, eager):
            lat, g, fs = upload(q, dims, U, psi, "F32")
            for f in fs:  # 20 different argument sets: 20 graphs
                q.smear(g, [f], 0.25, 3)
            q.smear(g, [fs[0]], 0.25, 3)  # the first graph was evicted: rebuilt
            res.append([q.read(f) for f in fs])
            free_all(q, [g] + fs)
        for a, b in zip(*res):
            assert np.array_equal(a, b)
    finally:
        eager.close()


def test_batch_equals_single_bitwise(qdp):
    sizes = [(4, 4, 4, 8), (6, 6, 6, 4), (8, 4, 4, 2), (4, 4, 4, 8)]
    jobs, single, expect = [], [], []
    for j, dims in enumerate(sizes):
        U = synth.su3_links(dims, 4001 + j)
        src = synth.point_source(dims, range(12))
        lat, g, fs = upload(qdp, dims, U, src, "F32")
        _, g2, fs2 = upload(qdp, dims, U, src, "F32")
        jobs.append((g, fs, fs))
        single.append((g2, fs2))
        expect.append(oracle.smear(U, src[:2], dims, 0.25, 9))
    qdp.smear_batch(jobs, 0.25, 9)
    for (g2, fs2) in single:
        qdp.smear(g2, fs2, 0.25, 9)
    for (g, fs, _), (g2, fs2), ex in zip(jobs, single, expect):
        for c in range(12):
            assert np.array_equal(qdp.read(fs[c]), qdp.read(fs2[c]))
        for c in range(2):
            assert rel(qdp.read(fs[c]), ex[c]) <= 1e-5
        free_all(qdp, [g, g2] + fs + fs2)


def _device_equal(q, a, b):
    """Bitwise equality of two FERMION fields on the device: the FP64 sum of
    |a - b|^2 over all sites is exactly 0 only if every difference is 0."""
    d = q.sum_multi([("field", a), ("field", b), ("sub",), ("local_norm2",)], "all", 1, 1)
    return d[0, 0].real == 0.0


@pytest.mark.parametrize("shape", [(1, 1, 1, 2, 0, 0), (2, 2, 0, 0, 0, 0), (1, 1, 1, 2, 0, 1), (2, 2, 0, 0, 0, 1),
                                   None])
def test_batch_blocks_walk_across_lattices_bitwise(qdp, shape):
    """More work items than the persistent grid has blocks: the lattices hold
    over 10k (lattice, 64-site tile) items, above the most 64-thread blocks
    256 CUs can hold (32 waves each), so blocks take several items, and their
    later items lie in other lattices (zstack = 1: one block per item, the
    lattice found by a search over the item offsets).  Every column of every
    lattice must equal the one-lattice smearing bitwise; two columns of the
    small lattices are also checked against the oracle."""
    sizes = [(16, 16, 16, 32), (6, 6, 6, 4), (16, 16, 16, 32), (12, 12, 12, 24), (16, 16, 16, 32),
             (8, 8, 8, 16), (16, 16, 16, 32), (16, 16, 16, 32), (4, 4, 4, 8)]
    items = sum(2 * -(-synth.volume(d) // 2 // 64) for d in sizes)
    assert items > 256 * 32
    niter = 5
    if shape is not None:
        qdp.set_shape(*shape)
    try:
        jobs, single, small = [], [], []
        for j, dims in enumerate(sizes):
            lat = qdp.lattice(dims)
            g = qdp.alloc(lat, "GAUGE", "F32")
            qdp.fill_random_su3(g, 4101 + j)
            fs = [qdp.alloc(lat, "FERMION", "F32") for _ in range(12)]
            fs2 = [qdp.alloc(lat, "FERMION", "F32") for _ in range(12)]
            scale = (24.0 * synth.volume(dims)) ** -0.5
            for c, (f, f2) in enumerate(zip(fs, fs2)):
                qdp.fill_gaussian(f, 4201 + j, c, scale)
                qdp.fill_gaussian(f2, 4201 + j, c, scale)
            jobs.append((g, fs, fs))
            single.append((g, fs2))
            if synth.volume(dims) <= 4096:
                small.append((j, dims, fs))
        qdp.smear_batch(jobs, 0.25, niter)
        for g, fs2 in single:
            qdp.smear(g, fs2, 0.25, niter)
        for j, ((g, fs, _), (_, fs2)) in enumerate(zip(jobs, single)):
            for c in range(12):
                assert _device_equal(qdp, fs[c], fs2[c]), (j, c)
        for j, dims, fs in small:
            U = synth.su3_links(dims, 4101 + j)
            src = synth.gaussian_propagator(dims, 4201 + j, columns=[0, 11])
            ex = oracle.smear(U, src, dims, 0.25, niter)
            for k, c in enumerate((0, 11)):
                assert rel(qdp.read(fs[c]), ex[k]) <= 1e-5, (j, c)
    finally:
        qdp.set_shape(0)
        for g, fs, _ in jobs:
            free_all(qdp, [g] + fs)
        for _, fs2 in single:
            free_all(qdp, fs2)


def test_zero_iterations_copies(qdp):
    dims = (4, 4, 2, 2)
    psi = synth.gaussian_propagator(dims, 9, ncols=2)
    lat, g, fs = upload(qdp, dims, synth.su3_links(dims, 9), psi, "F64")
    outs = [qdp.alloc(lat, "FERMION", "F64") for _ in fs]
    qdp.smear_to(g, fs, outs, 0.25, 0)
    for o, c in zip(outs, psi):
        assert np.array_equal(qdp.read(o), c)
    free_all(qdp, [g] + fs + outs)


def test_smear_errors(qdp):
    from paper_1111_5596_amd.qdpmi import QdpError

    dims = (4, 4, 4, 4)
    lat = qdp.lattice(dims)
    g = qdp.alloc(lat, "GAUGE", "F32")
    f = qdp.alloc(lat, "FERMION", "F32")
    h = qdp.alloc(lat, "FERMION", "F64")
    other = qdp.alloc(qdp.lattice((4, 4, 4, 2)), "FERMION", "F32")
    with pytest.raises(QdpError, match="UNSUPPORTED"):
        qdp.smear(g, [h], 0.25, 1)
    with pytest.raises(QdpError, match="LATTICE"):
        qdp.smear(g, [other], 0.25, 1)
    with pytest.raises(QdpError, match="TYPE"):
        qdp.smear(f, [f], 0.25, 1)
    with pytest.raises(QdpError, match="UNSUPPORTED"):
        qdp.smear(g, [f], 0.25, 1, j_decay=2)
    with pytest.raises(QdpError, match="ALIAS"):
        qdp.smear(g, [f, f], 0.25, 1)
    with pytest.raises(QdpError, match="ARG"):
        qdp.smear(g, [f], 0.25, -1)
    free_all(qdp, [g, f, h, other])


def test_f16s_keeps_relative_precision_over_wide_range(qdp):
    """F16S keeps one scale per site record, so a field whose magnitude changes
    by many orders from site to site (a smeared point source decays that way)
    keeps its relative precision at every site.  Two Gaussian columns times
    10^u(x), u rising from -30 to 10 across the spatial box (about two orders
    per lattice step, plus a random half order per site), one smearing step
    at kappa 0.25,
    the oracle run on the stored F16S links and columns: at every site the
    error stays within 2^-10 of the site's local scale B(x) = m(x) + 3 kappa
    sum_h m(x + h) (m = largest component magnitude of a record; a link
    entry is at most 1 in magnitude): FP16 output rounding is 2^-11 of the
    record's largest value, and the common-scale FP32 sums lose only terms
    below 2^-24 of the largest.  The register kernel and the LDS-window
    kernel agree bitwise."""
    dims = (8, 8, 8, 4)
    V = synth.volume(dims)
    U = synth.su3_links(dims, 7)
    rng = np.random.default_rng(11)
    # lexicographic site order, x fastest
    x, y, z = (np.arange(V) % 8, (np.arange(V) // 8) % 8, (np.arange(V) // 64) % 8)
    u = -30.0 + 40.0 * (x + y + z) / 21.0
    cols = []
    for _ in range(2):
        c = rng.standard_normal((V, 4, 3)) + 1j * rng.standard_normal((V, 4, 3))
        cols.append(c * (10.0 ** (u + rng.uniform(-0.5, 0.5, V)))[:, None, None])
    results = []
    try:
        for shape in [(4, 1, 1, 2, 0, 0, 0), (1, 1, 1, 0, 0, 0, 2)]:
            qdp.set_shape(*shape)
            lat, g, fs = upload(qdp, dims, U, cols, "F16S")
            Ust = qdp.read(g)
            stored = [qdp.read(f) for f in fs]
            qdp.smear(g, fs, 0.25, 1)
            assert qdp.get_shape() == shape
            got = [qdp.read(f) for f in fs]
            free_all(qdp, [g] + fs)
            for s_in, s_out in zip(stored, got):
                expect = oracle.smear_step(Ust, s_in, dims, 0.25)
                m = np.max(np.abs(s_in), axis=(1, 2))
                B = m.copy()
                for mu in range(3):
                    for sign in (1, -1):
                        B += 3 * 0.25 * oracle.shift(m[:, None], dims, mu, sign)[:, 0].real
                err = np.max(np.abs(s_out - expect), axis=(1, 2))
                assert np.all(err <= 2.0 ** -10 * B), float(np.max(err / B))
                # the local scales span the whole range: the bound is checked at
                # tiny and at large magnitudes alike
                assert B.min() < 1e-20 and B.max() > 1e5
            results.append(got)
    finally:
        qdp.set_shape(0)
    for a, b in zip(*results):
        assert np.array_equal(a, b)
