"""GPU parity at the benchmark configurations' full sizes, in the launch
configuration bench.py times (device-generated inputs, autotuned shapes,
graph replay).  The oracle computes sampled outputs: the smearing never
mixes time slices, so one slice of a column is an independent oracle
problem; the contraction of one slice is checked on the GPU's own smeared
slice.  Properties that hold at any size are checked on every slice."""

import numpy as np
import pytest

import oracle
from paper_1111_5596_amd import synth

pytestmark = pytest.mark.gpu

TOL = {"F32": 1e-5, "F16S": 2e-3}


@pytest.mark.parametrize("prec", ["F16S", "F32"])
def test_48cubed_96_smear_and_contract(qdp, prec):
    """48^3 x 96, links seed 5, 12-column Gaussian propagator seed 105, kappa
    0.25, N 100, even/odd passes, 16 bilinears."""
    from paper_1111_5596_amd import qdpmi

    dims = (48, 48, 48, 96)
    V = synth.volume(dims)
    sd = (48, 48, 48, 1)
    t = 37
    lat = qdp.lattice(dims)
    g = qdp.alloc(lat, "GAUGE", prec)
    qdp.fill_random_su3(g, 5)
    src = [qdp.alloc(lat, "FERMION", prec) for _ in range(12)]
    for j, f in enumerate(src):
        qdp.fill_gaussian(f, 105, j, (24.0 * V) ** -0.5)
    out = [qdp.alloc(lat, "FERMION", prec) for _ in range(12)]
    try:
        qdp.smear_to(g, src, out, 0.25, 100, mode=qdpmi.SMEAR_EVEN_ODD)
        C = qdp.contract(out, out)
        # sampled smearing parity: columns 0 and 7 on slice t, oracle from the
        # host generator's copy of the same inputs
        U = synth.su3_links(dims, 5, t_range=(t, t + 1))
        P = synth.gaussian_propagator(dims, 105, t_range=(t, t + 1), columns=[0, 7])
        ref = oracle.smear(U, P, sd, 0.25, 100)
        got_slices = {}
        for idx, j in enumerate([0, 7]):
            got = qdp.read_timeslices(out[j], t, t + 1)
            got_slices[j] = got
            err = np.linalg.norm(got - ref[idx]) / np.linalg.norm(ref[idx])
            assert err <= TOL[prec], (prec, j, err)
        # contraction parity on slice t, oracle on the GPU's smeared slice
        S = np.stack([qdp.read_timeslices(f, t, t + 1) for f in out])
        Cref = oracle.meson(S, S, sd)[:, 0]
        scale = abs(Cref[15].real)
        # F16S: FP32 colour sums of exact products of the stored halves
        assert np.max(np.abs(C[:, t] - Cref)) <= (2e-6 if prec == "F16S" else 1e-10) * scale
        # properties on every slice: C_15 > 0 real, |C_n| <= C_15, Im C_n ~ 0
        c15 = C[15].real
        assert np.all(c15 > 0)
        eps = 2e-6 if prec == "F16S" else 1e-9
        assert np.all(np.abs(C) <= c15[None, :] * (1 + eps))
        assert np.max(np.abs(C.imag)) <= eps * c15.max()
        # FP64 time-slice sums of |psi|^2 agree with C_15
        n2 = np.zeros(dims[3])
        for f in out:
            n2 += qdp.sum_multi([("field", f), ("local_norm2",)], "timeslice", 1, dims[3])[:, 0].real
        # F16S: C_15 from FP32 colour sums of the stored halves
        assert np.max(np.abs(n2 - c15) / c15) <= (2e-6 if prec == "F16S" else 1e-9)
    finally:
        for f in [g] + src + out:
            qdp.free(f)


def test_16cubed_32_point_source_pion_and_rho(qdp):
    """16^3 x 32, links seed 2, 12-column point source smeared (N 50), pion
    (n = 15) and rho (n = 1, 2, 4) from the smeared-smeared correlator; the
    oracle smears the whole source slice (point source: only slice 0 is
    non-zero)."""
    dims = (16, 16, 16, 32)
    sd = (16, 16, 16, 1)
    lat = qdp.lattice(dims)
    g = qdp.alloc(lat, "GAUGE", "F32")
    qdp.fill_random_su3(g, 2)
    cols = [qdp.alloc(lat, "FERMION", "F32") for _ in range(12)]
    for j, f in enumerate(cols):
        qdp.fill_point(f, 0, j // 3, j % 3)
    try:
        qdp.smear(g, cols, 0.25, 50)
        C = qdp.contract(cols, cols)
        U = synth.su3_links(dims, 2, t_range=(0, 1))
        Sref = oracle.smear(U, synth.point_source(sd, range(12)), sd, 0.25, 50)
        Cref = oracle.meson(Sref, Sref, sd)[:, 0]
        c15 = Cref[15].real
        for n in (15, 1, 2, 4):
            assert abs(C[n, 0] - Cref[n]) <= 1e-5 * c15, n
        assert np.count_nonzero(C[:, 1:]) == 0
        rho = np.mean([C[n, 0] for n in (1, 2, 4)])
        assert abs(rho - np.mean([Cref[n] for n in (1, 2, 4)])) <= 1e-5 * c15
    finally:
        for f in [g] + cols:
            qdp.free(f)


def test_16cubed_32_sink_smeared_synthetic_propagator(qdp):
    """16^3 x 32, links seed 2: the synthetic 12-column propagator (seed 102)
    sink-smeared with kappa 0.25, N 50 (FP32), pion (n = 15) and rho (n = 1,
    2, 4) correlators; the oracle smears slices 0 and 19 and contracts them."""
    dims = (16, 16, 16, 32)
    V = synth.volume(dims)
    sd = (16, 16, 16, 1)
    lat = qdp.lattice(dims)
    g = qdp.alloc(lat, "GAUGE", "F32")
    qdp.fill_random_su3(g, 2)
    cols = [qdp.alloc(lat, "FERMION", "F32") for _ in range(12)]
    for j, f in enumerate(cols):
        qdp.fill_gaussian(f, 102, j, (24.0 * V) ** -0.5)
    try:
        qdp.smear(g, cols, 0.25, 50, mode=1)
        C = qdp.contract(cols, cols)
        for t in (0, 19):
            U = synth.su3_links(dims, 2, t_range=(t, t + 1))
            P = synth.gaussian_propagator(dims, 102, t_range=(t, t + 1))
            Sref = oracle.smear(U, P, sd, 0.25, 50)
            got = np.stack([qdp.read_timeslices(f, t, t + 1) for f in cols])
            assert np.linalg.norm(got - Sref) <= 1e-5 * np.linalg.norm(Sref)
            Cref = oracle.meson(Sref, Sref, sd)[:, 0]
            c15 = Cref[15].real
            for n in (15, 1, 2, 4):
                assert abs(C[n, t] - Cref[n]) <= 1e-5 * c15, (t, n)
    finally:
        for f in [g] + cols:
            qdp.free(f)


def test_24cubed_48_chain_f16s_against_fp32_and_oracle(qdp):
    """24^3 x 48, links seed 3: source smearing of a 12-column point source
    (N 50), the synthetic propagator (seed 103) sink-smeared (N 50) and all 16
    bilinears, once with F16S storage and once with FP32 storage.  The oracle
    checks the smeared source on its slice, the smeared propagator and the
    correlators on slice 11; F16S and FP32 correlators agree to 2e-3 of
    C_15 on every slice."""
    dims = (24, 24, 24, 48)
    V = synth.volume(dims)
    sd = (24, 24, 24, 1)
    t = 11
    U_src = synth.su3_links(dims, 3, t_range=(0, 1))
    src_ref = oracle.smear(U_src, synth.point_source(sd, range(12)), sd, 0.25, 50)
    U = synth.su3_links(dims, 3, t_range=(t, t + 1))
    snk_ref = oracle.smear(U, synth.gaussian_propagator(dims, 103, t_range=(t, t + 1)), sd, 0.25, 50)
    C_ref = oracle.meson(snk_ref, snk_ref, sd)[:, 0]
    lat = qdp.lattice(dims)
    corr = {}
    for prec, tol in (("F32", 1e-5), ("F16S", 2e-3)):
        g = qdp.alloc(lat, "GAUGE", prec)
        qdp.fill_random_su3(g, 3)
        src = [qdp.alloc(lat, "FERMION", prec) for _ in range(12)]
        snk = [qdp.alloc(lat, "FERMION", prec) for _ in range(12)]
        try:
            for j, f in enumerate(src):
                qdp.fill_point(f, 0, j // 3, j % 3)
            qdp.smear(g, src, 0.25, 50, mode=1)
            got = np.stack([qdp.read_timeslices(f, 0, 1) for f in src])
            assert np.linalg.norm(got - src_ref) <= tol * np.linalg.norm(src_ref), prec
            # a reference zero stays an exact zero: every slice but the
            # source's has FP64 sum of squares exactly 0, in every column
            for j, f in enumerate(src):
                n2 = qdp.sum_multi([("field", f), ("local_norm2",)], "timeslice", 1, dims[3])[:, 0].real
                assert n2[0] > 0 and np.count_nonzero(n2[1:]) == 0, (prec, j)
            Csrc = qdp.contract(src, src)
            assert np.count_nonzero(Csrc[:, 1:]) == 0, prec
            for j, f in enumerate(snk):
                qdp.fill_gaussian(f, 103, j, (24.0 * V) ** -0.5)
            qdp.smear(g, snk, 0.25, 50, mode=1)
            got = np.stack([qdp.read_timeslices(f, t, t + 1) for f in snk])
            assert np.linalg.norm(got - snk_ref) <= tol * np.linalg.norm(snk_ref), prec
            C = qdp.contract(snk, snk)
            assert np.max(np.abs(C[:, t] - C_ref)) <= tol * C_ref[15].real, prec
            corr[prec] = C
        finally:
            for f in [g] + src + snk:
                qdp.free(f)
    c15 = corr["F32"][15].real
    assert np.max(np.abs(corr["F16S"] - corr["F32"]) / c15[None, :]) <= 2e-3


def test_batch_of_64_uneven_lattices(qdp):
    """64 lattices drawn from {8^3x16, 12^3x24, 16^3x32, 24^3x48}, links seed
    4001 + l, 12-column point sources, kappa 0.25, N 30, one persistent launch
    per iteration.  Every lattice's pion correlator on its source slice is
    checked against the oracle (the smearing never leaves the source slice,
    so that slice is the whole problem) and is exactly zero elsewhere; for the
    first lattice of each size and the last two of the work list, columns 0
    and 11 of the smeared source slice are compared element by element."""
    sizes = synth.lattice_sizes_batch()
    jobs, fields = [], []
    first_of = {}
    for l, dims in enumerate(sizes):
        lat = qdp.lattice(dims)
        g = qdp.alloc(lat, "GAUGE", "F32")
        qdp.fill_random_su3(g, 4001 + l)
        cols = [qdp.alloc(lat, "FERMION", "F32") for _ in range(12)]
        for j, f in enumerate(cols):
            qdp.fill_point(f, 0, j // 3, j % 3)
        jobs.append((g, cols, cols))
        fields.append((dims, g, cols))
        first_of.setdefault(dims, l)
    elementwise = set(first_of.values()) | {len(sizes) - 2, len(sizes) - 1}
    try:
        qdp.smear_batch(jobs, 0.25, 30)
        for l, (dims, g, cols) in enumerate(fields):
            C = qdp.contract(cols, cols, mask=1 << 15)
            assert np.count_nonzero(C[15, 1:]) == 0, l
            sd = dims[:3] + (1,)
            U = synth.su3_links(dims, 4001 + l, t_range=(0, 1))
            Sref = oracle.smear(U, synth.point_source(sd, range(12)), sd, 0.25, 30)
            ref = oracle.meson(Sref, Sref, sd)[15, 0].real
            assert abs(C[15, 0].real - ref) <= 1e-5 * ref, (l, dims)
            if l in elementwise:
                for j in (0, 11):
                    got = qdp.read_timeslices(cols[j], 0, 1)
                    err = np.linalg.norm(got - Sref[j]) / np.linalg.norm(Sref[j])
                    assert err <= 1e-5, (l, dims, j, err)
    finally:
        for dims, g, cols in fields:
            for f in [g] + cols:
                qdp.free(f)


def test_48cubed_96_hadron_contractions_sampled(qdp):
    """The benchmark's other contractions at full size, in its configuration:
    the 48^3 x 96 F16S Gaussian propagator (device generator, seed 105),
    mesons at four momenta (and, with a second propagator, seed 106, at zero
    and four momenta), the proton (both parities with u = d, and with a
    second propagator, seed 106, as d) and the Delta++, checked on time slice
    29 against the oracle run on that slice's stored values (the plane wave
    uses the spatial coordinates only, so a slice is an independent oracle
    problem).  Each lane of the baryon launch takes several sites here, so the
    per-site staging of the propagator in LDS is exercised repeatedly."""
    dims = (48, 48, 48, 96)
    V = synth.volume(dims)
    sd = (48, 48, 48, 1)
    t = 29
    lat = qdp.lattice(dims)
    cols = [qdp.alloc(lat, "FERMION", "F16S") for _ in range(12)]
    cols2 = [qdp.alloc(lat, "FERMION", "F16S") for _ in range(12)]
    try:
        for j in range(12):
            qdp.fill_gaussian(cols[j], 105, j, (24.0 * V) ** -0.5)
            qdp.fill_gaussian(cols2[j], 106, j, (24.0 * V) ** -0.5)
        S = np.stack([qdp.read_timeslices(f, t, t + 1) for f in cols])
        S2 = np.stack([qdp.read_timeslices(f, t, t + 1) for f in cols2])
        moms = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
        got = qdp.contract_mom(cols, cols, moms)[:, :, t]
        ref = oracle.meson_mom(S, S, sd, moms)[:, :, 0]
        # FP32 colour sums of exact products of the stored halves, FP64 after
        assert np.max(np.abs(got - ref)) <= 2e-6 * np.max(np.abs(ref))
        # two distinct propagators: the other meson kernels, zero and four momenta
        got = qdp.contract_mom(cols, cols2, moms)[:, :, t]
        ref = oracle.meson_mom(S, S2, sd, moms)[:, :, 0]
        assert np.max(np.abs(got - ref)) <= 2e-6 * np.max(np.abs(ref))
        got = qdp.contract(cols, cols2)[:, t]
        ref = oracle.meson(S, S2, sd)[:, 0]
        assert np.max(np.abs(got - ref)) <= 2e-6 * np.max(np.abs(ref))
        for parity in (1, -1):
            got = qdp.nucleon(cols, cols, parity=parity)[t]
            ref = oracle.nucleon(S, S, sd, parity)[0]
            assert abs(got - ref) <= 1e-10 * abs(ref), parity
        got = qdp.nucleon(cols, cols2)[t]
        ref = oracle.nucleon(S, S2, sd, 1)[0]
        assert abs(got - ref) <= 1e-10 * abs(ref)
        got = qdp.delta(cols)[t]
        ref = oracle.delta(S, sd, 1)[0]
        assert abs(got - ref) <= 1e-10 * abs(ref)
    finally:
        for f in cols + cols2:
            qdp.free(f)
