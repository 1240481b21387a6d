"""Benchmark: Jacobi smearing + meson contraction on one MI355X.

Workload (the largest single-GPU configuration): a 48^3 x 96 lattice
(10,616,832 sites), Haar-random SU(3) links (seed 5), a synthetic 12-column
Gaussian propagator (seed 105) of unit expected column norm; one step =
Jacobi smearing of all 12 columns, kappa = 0.25, N = 100 iterations, each
iteration two checkerboard passes (even sites, then odd sites, both reading
the previous iterate), followed by the 16-bilinear meson contraction with
FP64 products and time-slice sums.  Inputs are generated on the device by
the library's counter-based generator before timing and stay resident.

Headline (value): batched mixed precision -- FP16 storage of links and
spinors with per-record FP32 scales, FP32 arithmetic, all 12 columns per
launch, iterations replayed from a HIP graph.  Also reported: the same with
FP32 storage, and the plain FP32 path (one column at a time, the Jacobi
expression evaluated through qdp_eval, no graph, no column batching).

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
FLOP_PER_SITE_UPDATE = 1752


# Algorithmic HBM bytes per site-update used for the roofline (the
# measurement model of the workload definition): 12-column update, psi read
# and written once per iteration, links read twice per iteration on the
# checkerboard (once per subset).
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


def setup_fields(q, lat, prec, V):
    g = q.alloc(lat, "GAUGE", prec)
    q.fill_random_su3(g, LINK_SEED)
    src = [q.alloc(lat, "FERMION", prec) for _ in range(12)]
    for j, f in enumerate(src):
        q.fill_gaussian(f, PROP_SEED, j, 1.0 / (24.0 * V) ** 0.5)
    work = [q.alloc(lat, "FERMION", prec) for _ in range(12)]
    return g, src, work


def run_batched(q, torch, lat, prec, V, steps, warmup, mode=None):
    """Time `steps` full steps; returns a dict of timings and the correlator."""
    from paper_1111_5596_amd import qdpmi

    mode = qdpmi.SMEAR_EVEN_ODD if mode is None else mode
    g, src, work = setup_fields(q, lat, prec, V)
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
    for f in [g] + src + work:
        q.free(f)
    return {"wall_s": wall, "ms_per_step": 1e3 * wall / steps, "smear_ms": smear_ms,
            "contract_ms": contract_ms, "shape": shape, "corr": corr}


def run_plain(q, torch, lat, V):
    """Plain FP32 path: per column, per iteration, the Jacobi expression
    through qdp_eval on the even then the odd sites; then the contraction."""
    g, src, work = setup_fields(q, lat, "F32", V)
    tmp = q.alloc(lat, "FERMION", "F32")

    def jacobi(a):
        prog = [("field", a)]
        for i in range(3):
            prog += [("gauge", g, i), ("field", a), ("shift", i, 1), ("mul",),
                     ("real_const", KAPPA), ("mul",), ("add",)]
            prog += [("gauge", g, i), ("adj",), ("field", a), ("mul",), ("shift", i, -1),
                     ("real_const", KAPPA), ("mul",), ("add",)]
        return prog

    # one warm column-iteration, then the timed step
    q.eval(jacobi(src[0]), tmp, "even")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(12):
        a, b = src[j], work[j]
        q.eval([("field", a)], b)  # copy the source column
        for _ in range(NITER):
            q.eval(jacobi(b), tmp, "even")
            q.eval(jacobi(b), tmp, "odd")
            b, tmp = tmp, b
        if b != work[j]:  # odd iteration count: copy the result into work[j]
            q.eval([("field", b)], work[j])
            tmp = b
    corr = q.contract(work, work)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for f in set([g, tmp] + src + work):
        q.free(f)
    return {"wall_s": wall, "corr": corr}


def run_batch64(q, torch):
    """The multi-lattice workload: 64 lattices drawn from 8^3x16 .. 24^3x48,
    12-column point sources, kappa 0.25, N 30, FP32, one persistent launch per
    iteration, then the pion correlator of each lattice.  Returns
    (site-updates, seconds per step)."""
    from paper_1111_5596_amd import synth

    jobs, fields, su = [], [], 0
    for l, dims in enumerate(synth.lattice_sizes_batch()):
        lat = q.lattice(dims)
        g = q.alloc(lat, "GAUGE", "F32")
        q.fill_random_su3(g, 4001 + l)
        src = [q.alloc(lat, "FERMION", "F32") for _ in range(12)]
        for j, f in enumerate(src):
            q.fill_point(f, 0, j // 3, j % 3)
        dst = [q.alloc(lat, "FERMION", "F32") for _ in range(12)]
        jobs.append((g, src, dst))
        fields += [g] + src + dst
        su += 12 * dims[0] * dims[1] * dims[2] * dims[3] * 30
    q.smear_batch(jobs, KAPPA, 30)  # warm (graph build)
    for _, _, dst in jobs:
        q.contract(dst, dst, mask=1 << 15)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    q.smear_batch(jobs, KAPPA, 30)
    for _, _, dst in jobs:
        q.contract(dst, dst, mask=1 << 15)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for f in fields:
        q.free(f)
    return su, dt


def run_hadron_extras(q, torch, lat, V):
    """Wall time of the other hadron contractions on the same 48^3x96 F16S
    propagator (12 Gaussian columns): zero-momentum mesons, mesons at the
    four momenta (0,0,0), (1,0,0), (0,1,0), (0,0,1) in one launch, the proton
    and the Delta++ two-point functions.  Each call synchronises; the median
    of 3."""
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
    for f in cols:
        q.free(f)
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
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record(q.stream)
    for _ in range(reps):
        q.eval([("field", a)], b)
    e1.record(q.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    q.free(a)
    q.free(b)
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
    one per profiled launch shape, the first the shape of the profiled
    benchmark run) as dicts of their `key: value` lines."""
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


def measured_traffic(shape=None):
    """HBM bytes per launch of the profiled kernel (rocprofv3 FETCH_SIZE +
    WRITE_SIZE, scaled by the copy-kernel calibration) from a record taken on
    the current kernel sources and, when `shape` is given, with that launch
    shape; else None."""
    want = None if shape is None else ",".join(str(int(x)) for x in shape)
    for rec in traffic_records():
        if rec.get("kernel_source_sha256") != kernel_source_digest():
            continue
        if want is not None and rec.get("launch_shape_tuple") != want:
            continue
        try:
            return float(rec["traffic_bytes_per_launch"])
        except (KeyError, ValueError):
            continue
    return None


def cpu_baseline(full_steps_niter=NITER):
    """The FP64 oracle on one time slice (48^3 sites) of the same workload:
    12 columns smeared for 25 iterations (timed, scaled to N = 100) plus one
    contraction of the slice; threads = OMP_NUM_THREADS or all host cores."""
    import oracle
    from paper_1111_5596_amd import synth

    sample_dims = (48, 48, 48, 1)
    n_sample = 25
    U = synth.su3_links(DIMS, LINK_SEED, t_range=(0, 1))
    P = synth.gaussian_propagator(DIMS, PROP_SEED, t_range=(0, 1))
    t0 = time.perf_counter()
    S = oracle.smear(U, P, sample_dims, KAPPA, n_sample)
    t_smear = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.meson(S, S, sample_dims)
    t_meson = time.perf_counter() - t0
    vs = 48 ** 3
    step_time = t_smear * (full_steps_niter / n_sample) + t_meson
    rate = 12 * vs * full_steps_niter / step_time
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": rate, "unit": "site-updates/s", "cores": cores, "kind": "oracle",
            "sample": (f"one time slice (48^3 sites) of the 48^3x96 workload, 12 columns, FP64; "
                       f"smearing timed over {n_sample} iterations ({t_smear:.1f} s) and scaled to "
                       f"{full_steps_niter}, plus one 16-bilinear contraction ({t_meson:.1f} s)")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-storage batched run")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP32 path")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-lattice batch workload")
    ap.add_argument("--shape", default=None,
                    help="force the smearing launch shape site_waves,col_groups,xcd,waves_per_simd,flat "
                         "instead of autotuning (for profiler runs that must repeat a measured shape)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the smearing would shard by whole time slices with no exchange)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1111_5596_amd import qdpmi

    V = DIMS[0] * DIMS[1] * DIMS[2] * DIMS[3]
    q = qdpmi.Context(pool_bytes=72 << 30)
    if args.shape:
        q.set_shape(*[int(x) for x in args.shape.split(",")])
    lat = q.lattice(DIMS)
    site_updates = 12 * V * NITER
    launches = 2 * NITER

    print(f"[bench] F16S batched: {args.warmup} warmup + {args.steps} timed steps", file=sys.stderr, flush=True)
    f16 = run_batched(q, torch, lat, "F16S", V, args.steps, args.warmup)
    print(f"[bench] F16S step {f16['ms_per_step']:.1f} ms (smear {f16['smear_ms']:.1f} ms, "
          f"contract {f16['contract_ms']:.1f} ms)", file=sys.stderr, flush=True)
    fp32 = None
    if not args.no_fp32:
        fp32 = run_batched(q, torch, lat, "F32", V, max(1, args.steps // 2), 1)
        print(f"[bench] F32 step {fp32['ms_per_step']:.1f} ms", file=sys.stderr, flush=True)
    full = run_batched(q, torch, lat, "F16S", V, max(1, args.steps // 2), 1, mode=qdpmi.SMEAR_FULL)
    print(f"[bench] F16S full-update step {full['ms_per_step']:.1f} ms", file=sys.stderr, flush=True)
    batch = None
    if not args.no_batch:
        batch = run_batch64(q, torch)
        print(f"[bench] 64-lattice batch {batch[1] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    hadron = run_hadron_extras(q, torch, lat, V)
    print(f"[bench] hadron contractions {hadron}", file=sys.stderr, flush=True)
    plain = None
    if not args.no_plain:
        plain = run_plain(q, torch, lat, V)
        print(f"[bench] plain FP32 step {plain['wall_s'] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    copy_gbps, copy_bytes, copy_ms = copy_bandwidth(q, torch, lat)
    print(f"[bench] copy kernel {copy_gbps:.0f} GB/s ({copy_bytes / 1e9:.2f} GB in {copy_ms:.3f} ms)",
          file=sys.stderr, flush=True)
    q.close()

    value = site_updates / (f16["ms_per_step"] * 1e-3)
    launch_ms = f16["smear_ms"] / launches
    per_launch_units = 12 * V // 2  # site-updates of one checkerboard pass
    model_bytes = MODEL_BYTES_PER_SITE_UPDATE[("F16S", True)] * per_launch_units
    achieved = model_bytes / (launch_ms * 1e-3) / 1e9
    traffic = measured_traffic(f16["shape"])
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
        "config": {"workload": "48^3x96 Jacobi smearing kappa 0.25 N 100, 12 columns, even/odd passes, "
                               "FP16 storage + FP32 scales, FP32 arithmetic; 16-bilinear contraction, "
                               "FP64 products and sums",
                   "lattice": list(DIMS), "columns": 12, "iterations": NITER, "storage": "F16S",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": "smear_kernel<F16S> (one checkerboard subset pass, 12 columns)",
                     "bytes_per_launch": model_bytes, "units_per_launch": per_launch_units,
                     "bytes_per_unit": MODEL_BYTES_PER_SITE_UPDATE[("F16S", True)], "launch_ms": launch_ms,
                     "pass_minimum_bytes_per_launch": pass_bytes(V, "F16S", True),
                     "pass_minimum_GBps": pass_bytes(V, "F16S", True) / (launch_ms * 1e-3) / 1e9,
                     "pass_minimum_frac": pass_bytes(V, "F16S", True) / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS},
        "smear_ms_per_step": f16["smear_ms"],
        "contract_ms_per_step": f16["contract_ms"],
        "smear_site_updates_per_s": site_updates / (f16["smear_ms"] * 1e-3),
        "smear_tflops": site_updates * FLOP_PER_SITE_UPDATE / (f16["smear_ms"] * 1e-3) / 1e12,
        "launch_shape": list(f16["shape"]),
        "copy_kernel_GBps": copy_gbps,
        "frac_of_copy_bandwidth": achieved / copy_gbps,
    }
    out["f16s_full_update"] = {
        "value": site_updates / (full["ms_per_step"] * 1e-3), "ms_per_step": full["ms_per_step"],
        "smear_GBps_model": MODEL_BYTES_PER_SITE_UPDATE[("F16S", False)] * 12 * V / (full["smear_ms"] / NITER * 1e-3) / 1e9,
        "launch_shape": list(full["shape"])}
    out["hadron_contractions_48c96_f16s"] = hadron
    if batch:
        out["batch64_fp32"] = {"value": batch[0] / batch[1], "site_updates": batch[0], "ms": batch[1] * 1e3,
                               "workload": "64 lattices from {8^3x16,12^3x24,16^3x32,24^3x48}, 12 columns, "
                                           "N 30, one persistent launch per iteration + pion correlators"}
    if fp32:
        r32 = site_updates / (fp32["ms_per_step"] * 1e-3)
        l32 = fp32["smear_ms"] / launches
        out["fp32_batched"] = {"value": r32, "ms_per_step": fp32["ms_per_step"],
                               "smear_GBps": pass_bytes(V, "F32", True) / (l32 * 1e-3) / 1e9,
                               "launch_shape": list(fp32["shape"])}
        import numpy as np

        c16, c32 = f16["corr"], fp32["corr"]
        out["f16s_vs_fp32_correlator_err"] = float(np.max(np.abs(c16 - c32) / np.abs(c32[15].real)[None, :]))
    if plain:
        rp = site_updates / plain["wall_s"]
        out["plain_fp32"] = {"value": rp, "ms_per_step": plain["wall_s"] * 1e3}
        out["speedup_vs_plain_fp32"] = value / rp
        if fp32:
            out["fp32_batched_speedup_vs_plain"] = out["fp32_batched"]["value"] / rp
    if not args.no_cpu:
        print("[bench] oracle CPU baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
