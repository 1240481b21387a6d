"""Benchmark: Jacobi smearing + meson contraction on one MI355X.

Headline workload (the largest single-GPU configuration): a 48^3 x 96
lattice (10,616,832 sites), Haar-random SU(3) links (seed 5), a synthetic
12-column Gaussian propagator (seed 105) of unit expected column norm; one
step = Jacobi smearing of all 12 columns, kappa = 0.25, N = 100 iterations
on the checkerboard even and odd subsets (both read the previous iterate;
each iteration's two subset updates run as one launch, every workgroup
updating an even tile or the odd tile that holds its neighbours), followed
by the 16-bilinear meson contraction with FP64 products and time-slice sums.
Inputs are generated on the device by the library's counter-based generator
before timing and stay resident.

Headline (value): batched mixed precision -- FP16 storage of links and
spinors with per-record FP32 scales, FP32 arithmetic, all 12 columns per
launch, iterations replayed from a HIP graph.  Also reported: the same with
the two subsets as two launches per iteration, with FP32 storage, and the
plain FP32 path (one column at a time, the Jacobi expression evaluated
through qdp_eval on the even then the odd sites, no graph, no column
batching); the other workload configurations (4^3x8 plain method, 16^3x32
source and sink smearing with pion and rho, 24^3x48 FP16-storage chain with
all 16 bilinears, the 64-lattice batch); and, from the oracle leg, the
error of every result against the FP64 oracle on a sampled time slice.

Metric: smearing site-updates per second (site x 12-component column x
iteration) over the whole step, contraction included.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DIMS = (48, 48, 48, 96)
KAPPA = 0.25
NITER = 100
LINK_SEED, PROP_SEED = 5, 105
HBM_PEAK_GBPS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
FLOP_PER_SITE_UPDATE = 1752

# Algorithmic HBM bytes per site-update used for the roofline (the
# measurement model of the workload definition): 12-column update, psi read
# and written once per iteration, links read once per launch.  Key (storage,
# two launches per iteration): with the subsets as two launches the links are
# read twice per iteration.
MODEL_BYTES_PER_SITE_UPDATE = {("F32", True): 228, ("F16S", True): 124, ("F32", False): 210,
                               ("F16S", False): 114}


def pass_bytes(V: int, prec: str, checkerboard: bool) -> float:
    """Algorithmic HBM bytes of one smearing launch over all 12 columns.

    Full pass (every site updated): read psi at every site, write psi at
    every site, read the 3 spatial links at every site.  Checkerboard pass
    (one parity, V/2 sites): read psi at all V sites (own parity for the
    identity term, other parity as neighbours), write V/2 sites, read the
    3 spatial links at all V sites (U(x) on the own parity, U(x - i) on the
    other)."""
    col = {"F32": 96, "F16S": 52, "F64": 192}[prec]  # one 12-component column at one site
    link = {"F32": 72, "F16S": 40, "F64": 144}[prec]  # one colour matrix at one site
    if checkerboard:
        return V * (12 * col + 6 * col + 3 * link)
    return V * (24 * col + 3 * link)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def stream_timer(torch, q):
    """HIP events recorded on the library's stream (the one its kernels and
    graphs are launched on)."""
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def volume(dims):
    return dims[0] * dims[1] * dims[2] * dims[3]


def setup_gaussian(q, lat, dims, prec, link_seed, prop_seed):
    V = volume(dims)
    g = q.alloc(lat, "GAUGE", prec)
    q.fill_random_su3(g, link_seed)
    src = [q.alloc(lat, "FERMION", prec) for _ in range(12)]
    for j, f in enumerate(src):
        q.fill_gaussian(f, prop_seed, j, 1.0 / (24.0 * V) ** 0.5)
    work = [q.alloc(lat, "FERMION", prec) for _ in range(12)]
    return g, src, work


def setup_point(q, lat, prec, link_seed, ncols=12):
    g = q.alloc(lat, "GAUGE", prec)
    q.fill_random_su3(g, link_seed)
    src = [q.alloc(lat, "FERMION", prec) for _ in range(ncols)]
    for j, f in enumerate(src):
        q.fill_point(f, 0, j // 3, j % 3)
    work = [q.alloc(lat, "FERMION", prec) for _ in range(ncols)]
    return g, src, work


def free_all(q, fields):
    for f in fields:
        q.free(f)


def run_batched(q, torch, lat, prec, steps, warmup, mode, keep_slice=None):
    """Time `steps` headline steps (smear of the 12 columns + contraction).
    keep_slice = t: also return the GPU's smeared slice t (12 columns)."""
    V = volume(DIMS)
    g, src, work = setup_gaussian(q, lat, DIMS, prec, LINK_SEED, PROP_SEED)
    for _ in range(warmup):
        q.smear_to(g, src, work, KAPPA, NITER, mode=mode)
        q.contract(work, work)
    stream = q.stream
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    corr = None
    for k in range(steps):
        ev[k][0].record(stream)
        q.smear_to(g, src, work, KAPPA, NITER, mode=mode)
        ev[k][1].record(stream)
        corr = q.contract(work, work)  # synchronises: returns host data
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    smear_ms = sum(a.elapsed_time(b) for a, b, _ in ev) / steps
    contract_ms = sum(b.elapsed_time(c) for _, b, c in ev) / steps
    shape = q.get_shape()
    sl = None
    if keep_slice is not None:
        sl = [q.read_timeslices(f, keep_slice, keep_slice + 1) for f in work]
    free_all(q, [g] + src + work)
    return {"wall_s": wall, "ms_per_step": 1e3 * wall / steps, "smear_ms": smear_ms,
            "contract_ms": contract_ms, "shape": shape, "corr": corr, "slice": sl, "V": V}


def jacobi_program(g, a):
    """The Jacobi step psi + kappa sum_i [U_i psi(x+i) + U_i(x-i)^dag psi(x-i)]
    as a qdp_eval postfix program (the plain path)."""
    prog = [("field", a)]
    for i in range(3):
        prog += [("gauge", g, i), ("field", a), ("shift", i, 1), ("mul",),
                 ("real_const", KAPPA), ("mul",), ("add",)]
        prog += [("gauge", g, i), ("adj",), ("field", a), ("mul",), ("shift", i, -1),
                 ("real_const", KAPPA), ("mul",), ("add",)]
    return prog


def plain_smear(q, lat, g, src, work, niter, prec="F32"):
    """Plain path: per column, per iteration, the Jacobi expression through
    qdp_eval on the even then the odd sites (no graph, no batching).
    Returns the scratch field (the caller frees it)."""
    tmp = q.alloc(lat, "FERMION", prec)
    for j in range(len(src)):
        a, b = src[j], work[j]
        q.eval([("field", a)], b)  # copy the source column
        for _ in range(niter):
            q.eval(jacobi_program(g, b), tmp, "even")
            q.eval(jacobi_program(g, b), tmp, "odd")
            b, tmp = tmp, b
        if b != work[j]:  # odd iteration count: copy the result into work[j]
            q.eval([("field", b)], work[j])
            tmp = b
    return tmp


def run_plain(q, torch, lat):
    """Plain FP32 path on the headline workload, then the contraction."""
    g, src, work = setup_gaussian(q, lat, DIMS, "F32", LINK_SEED, PROP_SEED)
    # one warm column-iteration, then the timed step
    tmp0 = q.alloc(lat, "FERMION", "F32")
    q.eval(jacobi_program(g, src[0]), tmp0, "even")
    q.free(tmp0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tmp = plain_smear(q, lat, g, src, work, NITER)
    corr = q.contract(work, work)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    free_all(q, set([g, tmp] + src + work))
    return {"wall_s": wall, "corr": corr}


def run_config1(q, torch):
    """4^3 x 8 plain method: links seed 1, point source column 0, kappa
    0.25, N 10, FP64 and FP32, the Jacobi expression through qdp_eval, then
    C(t) = sum_x |psi(x, t)|^2 over the 8 slices (FP64 sums)."""
    dims = (4, 4, 4, 8)
    out = {}
    for prec in ("F64", "F32"):
        lat = q.lattice(dims)
        g, src, work = setup_point(q, lat, prec, 1, ncols=1)
        tmp = plain_smear(q, lat, g, src, work, 10, prec)
        psi = q.read(work[0])
        C = q.sum_multi([("field", work[0]), ("local_norm2",)], "timeslice", 1, dims[3])[:, 0].real
        out[prec] = {"psi": psi, "C": C}
        free_all(q, [g, tmp] + src + work)
    return out


def run_config2(q, torch):
    """16^3 x 32, links seed 2: source smearing of the 12-column point
    source (N 50) and sink smearing of the synthetic 12-column propagator
    (seed 102, N 50), FP32; pion (n = 15) and rho (n = 1, 2, 4) correlators
    of the sink-smeared propagator.  Batched path (12 columns per launch,
    HIP graph) and plain path, each timed over SRC + SNK + contraction."""
    dims, n = (16, 16, 16, 32), 50
    V = volume(dims)
    lat = q.lattice(dims)
    mask = (1 << 15) | (1 << 1) | (1 << 2) | (1 << 4)
    res = {}
    for path in ("batched", "plain"):
        gs, ps, ws = setup_point(q, lat, "F32", 2)
        _, pg, wg = setup_gaussian(q, lat, dims, "F32", 2, 102)
        free_all(q, [_])
        reps = 3 if path == "batched" else 1
        if path == "batched":  # warm: autotune and graph build
            q.smear_to(gs, ps, ws, KAPPA, n, mode=0)
            q.smear_to(gs, pg, wg, KAPPA, n, mode=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            if path == "batched":
                q.smear_to(gs, ps, ws, KAPPA, n, mode=0)
                q.smear_to(gs, pg, wg, KAPPA, n, mode=0)
            else:
                free_all(q, [plain_smear(q, lat, gs, ps, ws, n), plain_smear(q, lat, gs, pg, wg, n)])
            C = q.contract(wg, wg, mask=mask)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        res[path] = {"value": 2 * 12 * V * n / dt, "ms": dt * 1e3}
        if path == "batched":
            res["src_slice0"] = [q.read_timeslices(f, 0, 1) for f in ws]
            res["snk_slice0"] = [q.read_timeslices(f, 0, 1) for f in wg]
            res["C"] = C
        free_all(q, [gs] + ps + ws + pg + wg)
    return res


def run_config3(q, torch):
    """24^3 x 48, links seed 3: SRC (12-column point source, N 50) ->
    synthetic propagator (seed 103) -> SNK (N 50) -> all 16 bilinears, F16S
    storage and FP32 storage (FP64 products and sums), fused even/odd
    launches.  Returns rates, the F16S launch duration and slice-0 data."""
    dims, n = (24, 24, 24, 48), 50
    V = volume(dims)
    lat = q.lattice(dims)
    res = {}
    for prec in ("F16S", "F32"):
        gs, ps, ws = setup_point(q, lat, prec, 3)
        _, pg, wg = setup_gaussian(q, lat, dims, prec, 3, 103)
        free_all(q, [_])
        q.smear_to(gs, ps, ws, KAPPA, n, mode=0)  # warm
        q.smear_to(gs, pg, wg, KAPPA, n, mode=0)
        torch.cuda.synchronize()
        e0, e1 = stream_timer(torch, q)
        reps = 3
        t0 = time.perf_counter()
        e0.record(q.stream)
        for _ in range(reps):
            q.smear_to(gs, ps, ws, KAPPA, n, mode=0)
            q.smear_to(gs, pg, wg, KAPPA, n, mode=0)
        e1.record(q.stream)
        C = q.contract(wg, wg)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        smear_ms = e0.elapsed_time(e1) / reps
        res[prec] = {"value": 2 * 12 * V * n / dt, "ms": dt * 1e3, "smear_ms": smear_ms,
                     "launch_ms": smear_ms / (2 * n), "shape": list(q.get_shape()),
                     "src_slice0": [q.read_timeslices(f, 0, 1) for f in ws],
                     "snk_slice0": [q.read_timeslices(f, 0, 1) for f in wg], "C": C}
        free_all(q, [gs] + ps + ws + pg + wg)
    return res


def run_batch64(q, torch, reps=3):
    """The multi-lattice workload: 64 lattices drawn from 8^3x16 .. 24^3x48,
    12-column point sources, kappa 0.25, N 30, FP32, one launch over all the
    lattices per iteration replayed from a HIP graph; then the pion correlator of each
    lattice.  The smearing is timed with HIP events on the library's stream
    (median of `reps` replays), the 64 contractions separately."""
    from paper_1111_5596_amd import synth

    jobs, fields, su, sizes = [], [], 0, []
    for l, dims in enumerate(synth.lattice_sizes_batch()):
        lat = q.lattice(dims)
        g, src, dst = setup_point(q, lat, "F32", 4001 + l)
        jobs.append((g, src, dst))
        fields += [g] + src + dst
        su += 12 * volume(dims) * 30
        sizes.append(dims)
    q.smear_batch(jobs, KAPPA, 30)  # warm (autotune, graph build)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = stream_timer(torch, q)
        e0.record(q.stream)
        q.smear_batch(jobs, KAPPA, 30)
        e1.record(q.stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    smear_ms = sorted(ts)[len(ts) // 2]
    t0 = time.perf_counter()
    C15 = [q.contract(dst, dst, mask=1 << 15)[15].real for _, _, dst in jobs]
    contract_ms = (time.perf_counter() - t0) * 1e3
    # slice 0 of columns 0 and 7 of the first lattice of each size and of
    # the last two lattices of the list, for the oracle comparison
    pick = sorted(set([sizes.index(d) for d in set(sizes)] + [len(jobs) - 2, len(jobs) - 1]))
    slices = {l: [q.read_timeslices(jobs[l][2][j], 0, 1) for j in (0, 7)] for l in pick}
    shape = q.get_shape()
    free_all(q, fields)
    return {"site_updates": su, "smear_ms": smear_ms, "smear_ms_all": ts, "contract_ms": contract_ms,
            "C15": C15, "sizes": sizes, "slices": slices, "shape": list(shape)}


def run_hadron_extras(q, torch, lat):
    """Wall time of the other hadron contractions on the same 48^3x96 F16S
    propagator (12 Gaussian columns): zero-momentum mesons, mesons at the
    four momenta (0,0,0), (1,0,0), (0,1,0), (0,0,1) in one launch, the proton
    and the Delta++ two-point functions.  Each call synchronises; the median
    of 3."""
    V = volume(DIMS)
    cols = [q.alloc(lat, "FERMION", "F16S") for _ in range(12)]
    for j, f in enumerate(cols):
        q.fill_gaussian(f, 105, j, (24.0 * V) ** -0.5)
    moms = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    calls = {"meson_p0_ms": lambda: q.contract(cols, cols),
             "meson_4mom_ms": lambda: q.contract_mom(cols, cols, moms),
             "nucleon_ms": lambda: q.nucleon(cols, cols),
             "delta_pp_ms": lambda: q.delta(cols)}
    out = {}
    for name, fn in calls.items():
        fn()
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            ts.append((time.perf_counter() - t0) * 1e3)
        out[name] = sorted(ts)[1]
    free_all(q, cols)
    # rooflines on the wall times (launch, finish pass and the synchronising
    # copy of the result included): the mesons read the 12 F16S columns once
    # (52 B per site and column); the baryons are FP64 work, 2016 complex
    # multiply-adds (8 flop each) per site: nine colour steps of two pair
    # terms, each two 16-term inner products and two 40-term exchange traces
    meson_bytes = 12 * 52 * V
    baryon_flop = 2016 * 8 * V
    rl = {}
    for name in ("meson_p0_ms", "meson_4mom_ms"):
        gbps = meson_bytes / (out[name] * 1e-3) / 1e9
        rl[name[:-3]] = {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": gbps / HBM_PEAK_GBPS, "bytes": meson_bytes}
    for name in ("nucleon_ms", "delta_pp_ms"):
        tf = baryon_flop / (out[name] * 1e-3) / 1e12
        rl[name[:-3]] = {"bound": "fp64 vector", "achieved": tf, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tf / FP64_VECTOR_PEAK_TFLOPS, "flop": baryon_flop}
    out["roofline"] = rl
    return out


def copy_bandwidth(q, torch, lat):
    """Device copy of one F32 fermion field (qdp_eval dest = src): the plain
    copy kernel used to scale the HBM counters and as the attainable
    bandwidth reference."""
    a = q.alloc(lat, "FERMION", "F32")
    b = q.alloc(lat, "FERMION", "F32")
    q.fill_gaussian(a, 1, 0, 1.0)
    q.eval([("field", a)], b)
    nbytes = 2 * q.info(a).bytes
    e0, e1 = stream_timer(torch, q)
    reps = 20
    e0.record(q.stream)
    for _ in range(reps):
        q.eval([("field", a)], b)
    e1.record(q.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    free_all(q, [a, b])
    return nbytes / (ms * 1e-3) / 1e9, nbytes, ms


def kernel_source_digest() -> str:
    """Hash of the device code of the profiled smearing kernel: the kernel
    part of smear.hip (everything before its host driver) and the device
    headers it includes."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1111_5596_amd", "csrc")
    with open(os.path.join(csrc, "smear.hip"), "rb") as f:
        text = f.read()
    h.update(text[:text.index(b"// Host driver")])
    for name in ("device.hpp", "common.hpp"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_records():
    """The committed traffic records (profiles/smear_f16s_48c96_traffic*.txt,
    one per profiled launch mode and shape) as dicts of their `key: value`
    lines."""
    import glob

    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "smear_f16s_48c96_traffic*.txt")),
                   key=lambda p: (not p.endswith("_traffic.txt"), p))
    recs = []
    for path in paths:
        rec = {}
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    rec[k.strip()] = v.strip()
        recs.append(rec)
    return recs


def measured_traffic(shape=None, mode="full"):
    """HBM bytes per launch of the profiled kernel (rocprofv3 FETCH_SIZE +
    WRITE_SIZE, scaled by the copy-kernel calibration) from a record taken on
    the current kernel sources in launch mode `mode` ("full": both subsets
    in one launch, "even_odd": one subset per launch) and, when `shape` is
    given, with that launch shape; else None."""
    want = None if shape is None else ",".join(str(int(x)) for x in shape)
    for rec in traffic_records():
        if rec.get("kernel_source_sha256") != kernel_source_digest():
            continue
        if rec.get("launch_mode", "even_odd") != mode:
            continue
        if want is not None and rec.get("launch_shape_tuple") != want:
            continue
        try:
            return float(rec["traffic_bytes_per_launch"])
        except (KeyError, ValueError):
            continue
    return None


def smear_kernel_name(shape):
    """The smearing kernel a launch shape (site_waves, col_groups, xcd,
    waves_per_simd, flat, zstack, lds) runs on a whole F16S lattice."""
    lds = int(shape[6]) if len(shape) > 6 else 0
    return f"smear_lds_kernel<{lds}>" if lds else "smear_kernel"


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def relerr(got, ref):
    import numpy as np

    got, ref = np.asarray(got), np.asarray(ref)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def corr_err(got, ref):
    """max_n |C_n(t) - C_n,ref(t)| / C_15,ref(t) over the given slices."""
    import numpy as np

    got, ref = np.asarray(got), np.asarray(ref)
    return float(np.max(np.abs(got - ref) / np.abs(ref[15].real)))


def oracle_leg(res):
    """The FP64 oracle on the host cores: timed on one time slice (48^3
    sites) of the headline workload (12 columns, N = 100, plus the 16-bilinear
    contraction of the slice), and, from the same runs and a few more sampled
    slices, the error of every GPU result against it.  Smearing never mixes
    time slices, so a slice is an independent oracle problem."""
    import numpy as np

    import oracle
    from paper_1111_5596_amd import synth

    errs, per_config = {}, {}
    # config 5: slice 0 of the headline workload, N = 100 (timed)
    sd = (48, 48, 48, 1)
    U = synth.su3_links(DIMS, LINK_SEED, t_range=(0, 1))
    P = synth.gaussian_propagator(DIMS, PROP_SEED, t_range=(0, 1))
    t0 = time.perf_counter()
    S = oracle.smear(U, P, sd, KAPPA, NITER)
    t_smear = time.perf_counter() - t0
    t0 = time.perf_counter()
    Cref = oracle.meson(S, S, sd)
    t_meson = time.perf_counter() - t0
    vs = 48 ** 3
    rate = 12 * vs * NITER / (t_smear + t_meson)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    c5 = {}
    for key, r in res["c5"].items():
        if r is None or r.get("slice") is None:
            continue
        c5[key] = {"field_relL2": relerr(np.stack(r["slice"]), S),
                   "correlator_err": corr_err(r["corr"][:, :1], Cref)}
    errs["c5_48c96_slice0"] = c5
    base = {"value": rate, "unit": "site-updates/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": (f"one time slice (48^3 sites) of the 48^3x96 workload, 12 columns, FP64, N = {NITER} "
                       f"({t_smear:.1f} s), plus one 16-bilinear contraction of the slice ({t_meson:.2f} s)")}

    # config 1: the whole 4^3 x 8 lattice
    if res.get("c1"):
        d1 = (4, 4, 4, 8)
        U1 = synth.su3_links(d1, 1)
        p1 = synth.point_source(d1, [0])
        t0 = time.perf_counter()
        s1 = oracle.smear(U1, p1, d1, KAPPA, 10)[0]
        per_config["c1_4c8"] = {"value": volume(d1) * 10 / (time.perf_counter() - t0),
                                "sample": "whole lattice, 1 column, N = 10"}
        C1 = np.array([np.sum(np.abs(s1[t * 64:(t + 1) * 64]) ** 2) for t in range(8)])
        errs["c1_4c8"] = {prec: {"field_relL2": relerr(r["psi"], s1),
                                 "C_rel": float(np.max(np.abs(r["C"] - C1)) / C1[0]),
                                 "zeros_off_source_slice_exact": bool(np.all(r["C"][1:] == 0))}
                          for prec, r in res["c1"].items()}
    # configs 2 and 3: SRC (point source: only slice 0 is non-zero) and SNK on slice 0
    for key, dims, seed, n in (("c2", (16, 16, 16, 32), 2, 50), ("c3", (24, 24, 24, 48), 3, 50)):
        r = res.get(key)
        if not r:
            continue
        sdim = dims[:3] + (1,)
        Us = synth.su3_links(dims, seed, t_range=(0, 1))
        Ps = synth.gaussian_propagator(dims, 100 + seed, t_range=(0, 1))
        t0 = time.perf_counter()
        src = oracle.smear(Us, synth.point_source(sdim), sdim, KAPPA, n)
        snk = oracle.smear(Us, Ps, sdim, KAPPA, n)
        Cs = oracle.meson(snk, snk, sdim)
        per_config[f"{key}_{dims[0]}c{dims[3]}"] = {
            "value": 2 * 12 * volume(sdim) * n / (time.perf_counter() - t0),
            "sample": f"time slice 0: SRC + SNK smearing (2 x 12 columns, N = {n}) + one 16-bilinear contraction"}
        runs = {"F32": r["batched"]} if key == "c2" else {p: r[p] for p in ("F16S", "F32")}
        if key == "c2":
            runs["F32"] = dict(runs["F32"], src_slice0=r["src_slice0"], snk_slice0=r["snk_slice0"], C=r["C"])
        out = {}
        for prec, rr in runs.items():
            C = rr["C"][:, :1]
            mask = [1, 2, 4, 15] if key == "c2" else list(range(16))
            out[prec] = {"src_field_relL2": relerr(np.stack(rr["src_slice0"]), src),
                         "snk_field_relL2": relerr(np.stack(rr["snk_slice0"]), snk),
                         "correlator_err": float(np.max(np.abs(C[mask] - Cs[mask]) / abs(Cs[15, 0].real)))}
        errs[f"{key}_slice0"] = out
    # config 4: every lattice's pion C_15(t = 0) on its source slice, and the
    # field on slice 0 of two columns for the sampled lattices
    b = res.get("c4")
    if b:
        c15_err, field_err = 0.0, 0.0
        cache = {}
        t_c4, u_c4 = 0.0, 0
        for l, dims in enumerate(b["sizes"]):
            sdim = dims[:3] + (1,)
            Ul = synth.su3_links(dims, 4001 + l, t_range=(0, 1))
            t0 = time.perf_counter()
            Sl = oracle.smear(Ul, synth.point_source(sdim), sdim, KAPPA, 30)
            t_c4 += time.perf_counter() - t0
            u_c4 += 12 * volume(sdim) * 30
            c15 = float(np.sum(np.abs(Sl) ** 2))
            c15_err = max(c15_err, abs(b["C15"][l][0] - c15) / c15)
            if l in b["slices"]:
                field_err = max(field_err, max(relerr(b["slices"][l][i], Sl[j]) for i, j in enumerate((0, 7))))
            cache[l] = c15
        zeros = all(np.all(np.asarray(c)[1:] == 0) for c in b["C15"])
        errs["c4_batch64"] = {"C15_t0_rel_max_over_64": c15_err, "field_relL2_sampled": field_err,
                              "zeros_off_source_slice_exact": bool(zeros)}
        per_config["c4_batch64"] = {"value": u_c4 / t_c4,
                                    "sample": "time slice 0 of each of the 64 lattices, 12 columns, N = 30"}
    if per_config:
        base["per_config"] = per_config
    return base, errs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-storage headline workload")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP32 path")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg (CPU baseline and errors)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-lattice batch workload")
    ap.add_argument("--no-configs", action="store_true", help="skip the 4^3x8, 16^3x32 and 24^3x48 workloads")
    ap.add_argument("--no-two-pass", action="store_true", help="skip the two-launch even/odd variant")
    ap.add_argument("--shape", default=None,
                    help="force the smearing launch shape site_waves,col_groups,xcd,waves_per_simd,flat,zstack[,lds] "
                         "instead of autotuning (for profiler runs that must repeat a measured shape)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the smearing would shard by whole time slices with no exchange)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1111_5596_amd import qdpmi

    V = volume(DIMS)
    q = qdpmi.Context(pool_bytes=72 << 30)
    if args.shape:
        q.set_shape(*[int(x) for x in args.shape.split(",")])
    lat = q.lattice(DIMS)
    site_updates = 12 * V * NITER
    FULL, EO = qdpmi.SMEAR_FULL, qdpmi.SMEAR_EVEN_ODD
    want_slice = None if args.no_cpu else 0

    log(f"F16S fused even/odd: {args.warmup} warmup + {args.steps} timed steps")
    f16 = run_batched(q, torch, lat, "F16S", args.steps, args.warmup, FULL, keep_slice=want_slice)
    log(f"F16S step {f16['ms_per_step']:.1f} ms (smear {f16['smear_ms']:.1f} ms, contract {f16['contract_ms']:.1f} ms)")
    two = None
    if not args.no_two_pass:
        two = run_batched(q, torch, lat, "F16S", max(1, args.steps // 2), 1, EO, keep_slice=want_slice)
        log(f"F16S two launches per iteration: step {two['ms_per_step']:.1f} ms")
    fp32 = None
    if not args.no_fp32:
        fp32 = run_batched(q, torch, lat, "F32", max(1, args.steps // 2), 1, FULL, keep_slice=want_slice)
        log(f"F32 step {fp32['ms_per_step']:.1f} ms")
    res = {"c5": {"F16S": f16, "F16S_two_launch": two, "F32": fp32}}
    batch = None
    if not args.no_batch:
        batch = run_batch64(q, torch)
        res["c4"] = batch
        log(f"64-lattice batch: smear {batch['smear_ms']:.1f} ms, contractions {batch['contract_ms']:.1f} ms")
    if not args.no_configs:
        res["c1"] = run_config1(q, torch)
        res["c2"] = run_config2(q, torch)
        log(f"16^3x32: batched {res['c2']['batched']['ms']:.1f} ms, plain {res['c2']['plain']['ms']:.1f} ms")
        res["c3"] = run_config3(q, torch)
        log(f"24^3x48: F16S {res['c3']['F16S']['ms']:.1f} ms, F32 {res['c3']['F32']['ms']:.1f} ms")
    hadron = run_hadron_extras(q, torch, lat)
    log(f"hadron contractions { {k: v for k, v in hadron.items() if k != 'roofline'} }")
    plain = None
    if not args.no_plain:
        plain = run_plain(q, torch, lat)
        log(f"plain FP32 step {plain['wall_s'] * 1e3:.1f} ms")
    copy_gbps, copy_bytes, copy_ms = copy_bandwidth(q, torch, lat)
    log(f"copy kernel {copy_gbps:.0f} GB/s ({copy_bytes / 1e9:.2f} GB in {copy_ms:.3f} ms)")
    q.close()

    value = site_updates / (f16["ms_per_step"] * 1e-3)
    launch_ms = f16["smear_ms"] / NITER  # one launch per iteration
    per_launch_units = 12 * V  # site-updates of one launch (every site, 12 columns)
    bpu = MODEL_BYTES_PER_SITE_UPDATE[("F16S", False)]
    model_bytes = bpu * per_launch_units
    achieved = model_bytes / (launch_ms * 1e-3) / 1e9
    traffic = measured_traffic(f16["shape"], "full")
    out = {
        "metric": "smearing site-updates/s + achieved HBM GB/s; batched/mixed vs plain FP32",
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f16["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (device-generated Haar SU(3) links seed 5, Gaussian propagator seed 105)",
        "config": {"workload": "48^3x96 Jacobi smearing kappa 0.25 N 100, 12 columns, checkerboard even/odd "
                               "subsets (both subset updates of an iteration in one launch), FP16 storage + "
                               "FP32 scales, FP32 arithmetic; 16-bilinear contraction, FP64 products and sums",
                   "lattice": list(DIMS), "columns": 12, "iterations": NITER, "storage": "F16S",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": smear_kernel_name(f16["shape"]) + " (F16S, both checkerboard subsets in one launch, "
                               "12 columns)",
                     "bytes_per_launch": model_bytes, "units_per_launch": per_launch_units,
                     "bytes_per_unit": bpu, "launch_ms": launch_ms},
        "smear_ms_per_step": f16["smear_ms"],
        "contract_ms_per_step": f16["contract_ms"],
        "smear_site_updates_per_s": site_updates / (f16["smear_ms"] * 1e-3),
        "smear_tflops": site_updates * FLOP_PER_SITE_UPDATE / (f16["smear_ms"] * 1e-3) / 1e12,
        "launch_shape": list(f16["shape"]),
        "copy_kernel_GBps": copy_gbps,
        "frac_of_copy_bandwidth": achieved / copy_gbps,
    }
    if two:
        l2 = two["smear_ms"] / (2 * NITER)
        out["f16s_two_launches"] = {
            "value": site_updates / (two["ms_per_step"] * 1e-3), "ms_per_step": two["ms_per_step"],
            "launch_ms": l2,
            "GBps_model_124B": MODEL_BYTES_PER_SITE_UPDATE[("F16S", True)] * (12 * V // 2) / (l2 * 1e-3) / 1e9,
            "GBps_pass_minimum": pass_bytes(V, "F16S", True) / (l2 * 1e-3) / 1e9,
            "traffic": measured_traffic(two["shape"], "even_odd"),
            "launch_shape": list(two["shape"])}
    out["hadron_contractions_48c96_f16s"] = hadron
    if fp32:
        r32 = site_updates / (fp32["ms_per_step"] * 1e-3)
        l32 = fp32["smear_ms"] / NITER
        out["fp32_batched"] = {"value": r32, "ms_per_step": fp32["ms_per_step"], "launch_ms": l32,
                               "GBps_model_210B": MODEL_BYTES_PER_SITE_UPDATE[("F32", False)] * 12 * V
                               / (l32 * 1e-3) / 1e9,
                               "launch_shape": list(fp32["shape"])}
        import numpy as np

        c16, c32 = f16["corr"], fp32["corr"]
        out["f16s_vs_fp32_correlator_err"] = float(np.max(np.abs(c16 - c32) / np.abs(c32[15].real)[None, :]))
    if batch:
        bl = batch["smear_ms"] / 30
        mean_units = batch["site_updates"] / 30
        out["batch64_fp32"] = {
            "value": batch["site_updates"] / ((batch["smear_ms"] + batch["contract_ms"]) * 1e-3),
            "smear_site_updates_per_s": batch["site_updates"] / (batch["smear_ms"] * 1e-3),
            "smear_ms": batch["smear_ms"], "smear_ms_replays": batch["smear_ms_all"],
            "contract_ms_64": batch["contract_ms"], "site_updates": batch["site_updates"],
            "roofline": {"bytes_per_unit": MODEL_BYTES_PER_SITE_UPDATE[("F32", False)],
                         "units_per_launch": mean_units, "launch_ms": bl,
                         "achieved_GBps": MODEL_BYTES_PER_SITE_UPDATE[("F32", False)] * mean_units / (bl * 1e-3) / 1e9,
                         "frac": MODEL_BYTES_PER_SITE_UPDATE[("F32", False)] * mean_units / (bl * 1e-3) / 1e9
                         / HBM_PEAK_GBPS},
            "launch_shape": batch["shape"],
            "workload": "64 lattices from {8^3x16,12^3x24,16^3x32,24^3x48}, 12 columns, N 30, one launch per "
                        "iteration over all 64 lattices (median of 3 graph replays, HIP events) + 64 pion "
                        "correlators"}
    if "c2" in res:
        c2 = res["c2"]
        out["c2_16c32_fp32"] = {"batched": {"value": c2["batched"]["value"], "ms": c2["batched"]["ms"]},
                                "plain": {"value": c2["plain"]["value"], "ms": c2["plain"]["ms"]},
                                "speedup": c2["batched"]["value"] / c2["plain"]["value"],
                                "note": "SRC + SNK smearing (2 x 12 columns, N 50) + pion/rho; 340 MB working "
                                        "set, at the 256 MB Infinity Cache size: no HBM roofline"}
    if "c3" in res:
        c3 = res["c3"]
        V3 = volume((24, 24, 24, 48))
        b3 = MODEL_BYTES_PER_SITE_UPDATE[("F16S", False)] * 12 * V3
        ach3 = b3 / (c3["F16S"]["launch_ms"] * 1e-3) / 1e9
        out["c3_24c48"] = {p: {"value": c3[p]["value"], "ms": c3[p]["ms"], "launch_ms": c3[p]["launch_ms"],
                               "launch_shape": c3[p]["shape"]} for p in ("F16S", "F32")}
        out["c3_24c48"]["F16S"]["roofline"] = {"bytes_per_unit": MODEL_BYTES_PER_SITE_UPDATE[("F16S", False)],
                                               "units_per_launch": 12 * V3, "achieved_GBps": ach3,
                                               "frac": ach3 / HBM_PEAK_GBPS}
        out["c3_24c48"]["F16S_speedup_vs_F32"] = c3["F16S"]["value"] / c3["F32"]["value"]
    if plain:
        rp = site_updates / plain["wall_s"]
        out["plain_fp32"] = {"value": rp, "ms_per_step": plain["wall_s"] * 1e3}
        out["speedup_vs_plain_fp32"] = value / rp
        if fp32:
            out["fp32_batched_speedup_vs_plain"] = out["fp32_batched"]["value"] / rp
    if not args.no_cpu:
        log("oracle leg: CPU baseline and errors against the oracle")
        out["cpu_baseline"], out["oracle_error"] = oracle_leg(res)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
