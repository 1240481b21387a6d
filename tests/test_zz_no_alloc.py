"""GPU test of the allocation-free meson contraction
(qdp_hadron_contract_noalloc): its device output must equal, bitwise, what
qdp_hadron_contract returns for the same columns (same kernels, same
fixed-order sums), on two calls in a row, the second on a smaller lattice
(fewer time slices and partial sums than the first left in the shared
scratch array); both are also checked against the oracle within the
precision's tolerance.  Error paths are forced from the host: a spilled
column, and a lattice whose partial sums exceed the scratch array."""

import numpy as np
import pytest

import oracle
from paper_1111_5596_amd import synth

pytestmark = pytest.mark.gpu


def _cols(q, lat, S, prec):
    fs = []
    for c in S:
        f = q.alloc(lat, "FERMION", prec)
        q.write(f, c)
        fs.append(f)
    return fs


def _noalloc(q, torch, S1, S2, Lt, mask=0xFFFF, t0=0):
    out = torch.full((16 * Lt * 2,), float("nan"), dtype=torch.float64, device="cuda")
    q.contract_noalloc(S1, S2, out.data_ptr(), mask=mask, t0=t0)
    q.sync()
    return out.cpu().numpy().view(np.complex128).reshape(16, Lt)


def test_noalloc_matches_contract_two_calls(qdp):
    import torch

    cases = [((8, 8, 8, 16), "F32", 0xFFFF, 0, 301), ((4, 4, 4, 8), "F16S", (1 << 15) | (1 << 5) | 1, 3, 302)]
    for dims, prec, mask, t0, seed in cases:
        print(f"noalloc case dims={dims} prec={prec} mask={mask:#x} t0={t0}", flush=True)
        S1 = synth.gaussian_propagator(dims, seed)
        S2 = synth.gaussian_propagator(dims, seed + 50)
        lat = qdp.lattice(dims)
        a = _cols(qdp, lat, S1, prec)
        b = _cols(qdp, lat, S2, prec)
        Lt = dims[3]
        got = _noalloc(qdp, torch, a, b, Lt, mask, t0)
        want = qdp.contract(a, b, mask=mask, t0=t0)
        assert np.array_equal(got, want), float(np.max(np.abs(got - want)))
        # the oracle on the stored (rounded) inputs; products and sums are
        # FP64 (F16S: FP32 colour sums of exact products of the stored
        # halves), so only rounding order differs
        S1r = np.stack([qdp.read(f) for f in a])
        S2r = np.stack([qdp.read(f) for f in b])
        ref = np.roll(oracle.meson(S1r, S2r, dims), -t0, axis=1)
        tol = 2e-6 if prec == "F16S" else 1e-11
        for n in range(16):
            if mask & (1 << n):
                assert np.max(np.abs(got[n] - ref[n])) <= tol * np.max(np.abs(ref))
            else:
                assert np.all(got[n] == 0)
        for f in a + b:
            qdp.free(f)


def test_noalloc_refuses_spilled_column_and_oversized_scratch():
    import torch

    from paper_1111_5596_amd import qdpmi

    q = qdpmi.Context(pool_bytes=256 << 20, host_spill_bytes=64 << 20)
    try:
        dims = (4, 4, 4, 8)
        lat = q.lattice(dims)
        S = _cols(q, lat, synth.gaussian_propagator(dims, 303), "F32")
        q.evict(S[4])
        out = torch.zeros(16 * 8 * 2, dtype=torch.float64, device="cuda")
        with pytest.raises(qdpmi.QdpError) as ei:
            q.contract_noalloc(S, S, out.data_ptr())
        assert qdpmi.ERRORS[ei.value.status] == "QDP_ERR_STATE"
        assert "spilled" in str(ei.value)
        # 16386 slices of 2^3 sites: 256 * 16386 bytes of partial sums > 4 MiB
        big = q.lattice((2, 2, 2, 16386))
        B = [q.alloc(big, "FERMION", "F32") for _ in range(12)]
        outb = torch.zeros(16 * 16386 * 2, dtype=torch.float64, device="cuda")
        with pytest.raises(qdpmi.QdpError) as ei:
            q.contract_noalloc(B, B, outb.data_ptr())
        assert qdpmi.ERRORS[ei.value.status] == "QDP_ERR_UNSUPPORTED"
        assert "scratch" in str(ei.value)
        q.sync()
    finally:
        q.close()
