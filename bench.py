"""Throughput benchmark of the reconstruction hot path on one MI355X.

A step is one iteration of the EM-type algorithm (Alg. 5) on the 128 x 128
voxel x 64 q slice with a 128 x 128 detector: forward projection, Poisson
ratio and float64 data-fit terms, back projection, separable-surrogate update
and the float64 objective, all in the HIP library.  The metric counts the
nominal voxel*pixel*q evaluations of one forward plus one adjoint
(2 * 16384 * 16384 * 64 = 3.436e10) per step.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extras]
    python bench.py --workload batch64 [--steps K] [--warmup W]
    python bench.py --workload warm [--tto-cases N]
    python bench.py --workload os [--steps K]
    python bench.py --workload sai [--steps K] [--sai-interp linear|nearest]
    python bench.py --workload energy [--steps K]

Prints one JSON line.  The operators run in interval form by default (the
sum over q of a class read from per-voxel tables over the sorted spectrum-bin
thresholds); each reads its 8-byte class records once per call, so the
roofline entry is HBM-bound: algorithmic bytes per launch (class records,
the adjoint's per-group bin positions, the input and output arrays) over the
event-timed average duration of the dominant operator inside the timed
region, against 8 TB/s.  When the direct kernels run instead (the interval
form switched off or not applicable), the entry is VALU-bound with their work
model: 4 lane-ops per open in-band triple plus 60 per open pair and 10 per
pair on the fly, or 20 per class record of the factor store, against the
non-packed FP32 issue rate of the chip (an FMA-chain kernel's measured rate
beside it).  Wall times of the bench's phases are printed with the line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "slice128"
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9      # CUs x SIMDs x lanes x clock: 3.93e13 lane-ops/s
PEAK_HBM = 8.0e12                         # bytes/s
OPS_PER_TRIPLE, OPS_PER_OPEN_PAIR, OPS_PER_PAIR = 4.0, 60.0, 10.0
OPS_PER_RECORD = 20.0                     # factor store: unpack a class record, weights, band range
GOLDEN = os.path.join(ROOT, "tests", "golden")
SRC = [os.path.join(ROOT, "paper_1603_06400_amd", "csrc", n) for n in ("csx_ops.hip", "csx_interval.hip")]


def source_hash() -> str:
    """Hash of the operator sources' code (comments and whitespace removed), so
    that the stored counters follow code changes but not comment edits."""
    import re
    text = ""
    for path in ([SRC] if isinstance(SRC, str) else SRC):
        with open(path, encoding="utf-8") as fh:
            text += fh.read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    text = " ".join(text.split())
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def algorithmic_ops(census: dict, stored: bool = False, pairs_per_class: int = 4) -> float:
    """VALU lane-ops of one operator launch: the q loop's triples, plus the
    pair-factor work on the fly, or one class record per mirror class (4 pairs
    with the x -> -x mirror) read from the factor store."""
    if stored:
        return OPS_PER_TRIPLE * census["open_triples_in_band"] + OPS_PER_RECORD * census["pairs"] / pairs_per_class
    return (OPS_PER_TRIPLE * census["open_triples_in_band"] + OPS_PER_OPEN_PAIR * census["open_pairs"]
            + OPS_PER_PAIR * census["pairs"])


def interval_bytes(g, lr: bool) -> dict:
    """Algorithmic HBM bytes of one interval-form forward and adjoint launch.
    Forward: the 8-byte class records of every voxel group (the upper
    detector half's classes), the image and the detector.  Adjoint: the same
    records in interval order (padded to chunks of 8), the uint16 prefix-table
    index of every (node, bin edge) per group (rows of 72 entries when ne <= 64
    and nq <= 128, else ne + 1 rounded up to 8), one position-mask byte per
    chunk, the detector and the image."""
    groups = g.nz * (g.nx // 2) if lr else g.nz * g.nx
    slots = g.ndx * (g.ndy // 2)
    rstride = (slots + 7) // 8 * 8
    es = 72 if (g.ne <= 64 and g.nq <= 128) else (g.ne + 1 + 7) // 8 * 8
    records = 8.0 * groups * slots
    image, det = 4.0 * g.nvox * g.nq, 4.0 * g.npix
    records_a = 8.0 * groups * rstride
    positions = 2.0 * groups * g.nq * es + 1.0 * groups * (rstride // 8)
    return {"forward": records + image + det, "adjoint": records_a + positions + det + image,
            "records": records, "positions": positions}


def stored_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_slice128.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def cpu_baseline(g, f, y, n_pix=12288, n_vox=12288, one_core_div=16):
    """The FP64 oracle on a bounded sample of the same workload: forward at
    n_pix sampled pixels and adjoint at n_vox sampled voxels on every host
    thread, then on one thread with a sample one_core_div times smaller."""
    import oracle
    o = oracle.Oracle(g)
    rng = np.random.Generator(np.random.PCG64(5))
    cores = oracle.max_threads()

    def timed(npx, nvx):
        pix = rng.choice(g.npix, npx, replace=False)
        vox = rng.choice(g.nvox, nvx, replace=False)
        t0 = time.perf_counter()
        o.forward_pixels(f, pix)
        t1 = time.perf_counter()
        o.adjoint_voxels(y, vox)
        t2 = time.perf_counter()
        return (npx + nvx) * g.nvox * g.nq, t1 - t0, t2 - t1   # each sampled output sums over the other side

    evals, tf, ta = timed(n_pix, n_vox)
    oracle.set_threads(1)
    try:
        e1, tf1, ta1 = timed(n_pix // one_core_div, n_vox // one_core_div)
    finally:
        oracle.set_threads(cores)
    return {"value": evals / (tf + ta), "unit": "evals/s", "cores": cores,
            "kind": "oracle", "host": host_info(), "slice32": oracle_slice32(),
            "sample": f"FP64 oracle: forward at {n_pix} random pixels + adjoint at {n_vox} random "
                      f"voxels of the {WORKLOAD} workload ({evals:.3e} evals, "
                      f"{tf:.1f} s + {ta:.1f} s)",
            "one_core": {"value": e1 / (tf1 + ta1), "unit": "evals/s", "cores": 1,
                         "sample": f"forward at {n_pix // one_core_div} + adjoint at "
                                   f"{n_vox // one_core_div} random outputs ({e1:.3e} evals, "
                                   f"{tf1:.1f} s + {ta1:.1f} s)"}}


def host_info() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


def oracle_slice32() -> dict:
    """The FP64 oracle on the whole 32^2 x 32q slice: one forward, one adjoint
    and the 20-iteration Alg. 5 run from the uniform start, on every host
    thread."""
    import oracle
    from paper_1603_06400_amd import inputs
    w = inputs.workload("slice32")
    z = np.load(os.path.join(GOLDEN, "slice32_counts.npz"))
    g = w.geom.with_(C=float(z["C"]))
    y = z["y"].astype(np.float64)
    o = oracle.Oracle(g)
    f = inputs.phantom(w.geom, w.phantom_seed, w.n_rect)
    t0 = time.perf_counter()
    o.forward(f)
    t1 = time.perf_counter()
    o.adjoint(y)
    t2 = time.perf_counter()
    f0 = oracle.uniform_start(y, o.sensitivity())
    t3 = time.perf_counter()
    _, J = o.recon(y, None, f0, w.n_iter, w.beta)
    t4 = time.perf_counter()
    return {"forward_s": t1 - t0, "adjoint_s": t2 - t1, "recon_iters": w.n_iter,
            "recon_s": t4 - t3, "J_last": float(J[-1]),
            "evals_per_s": 2.0 * g.nvox * g.npix * g.nq / (t2 - t0)}


def gpu_slice32(reps: int = 5) -> dict:
    """The library on the same 32^2 x 32q slice: the 20-iteration Alg. 5 run
    from the uniform start (uniform start and objectives included), median of
    reps runs."""
    import torch
    from paper_1603_06400_amd import csx, inputs
    w = inputs.workload("slice32")
    z = np.load(os.path.join(GOLDEN, "slice32_counts.npz"))
    g = w.geom.with_(C=float(z["C"]))
    geo = csx.Geometry(g)
    y = torch.tensor(z["y"], dtype=torch.float32, device="cuda")
    f = geo.new_image()
    geo.recon(y, f, w.n_iter, w.beta)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = geo.recon(y, f, w.n_iter, w.beta)
        ts.append(time.perf_counter() - t0)
    return {"recon_iters": w.n_iter, "recon_ms_median": float(np.median(ts)) * 1e3, "J_last": float(J[-1])}


def operator_medians(geo, f, y, warm: int = 5, n: int = 50) -> dict:
    """Forward and adjoint launches one at a time, each bracketed by HIP
    events on the stream they run on: warm-ups, then the median of n."""
    import torch
    gbuf, bbuf = geo.new_detector(), geo.new_image()
    out = {"warmup": warm, "n": n}
    for name, fn in (("forward_ms", lambda: geo.forward(f, gbuf)), ("adjoint_ms", lambda: geo.backproject(y, bbuf))):
        for _ in range(warm):
            fn()
        ev = []
        for _ in range(n):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            ev.append((e0, e1))
        torch.cuda.synchronize()
        out[name] = float(np.median([a.elapsed_time(b) for a, b in ev]))
    return out


def bench_batch(args):
    """The batched form: 64 scans of uneven sizes (N in {48, 64, 96, 128}, nq in
    {32, 64}), launch shapes from the autotuner, reconstructed together by one
    replayed iteration graph; timed against the same scans run one after the
    other through the single-scan entry point.  Counts are Poisson draws around
    the library's own forward of each phantom, scaled to a maximum mean of 1e4."""
    import torch

    from paper_1603_06400_amd import autotune, csx, inputs

    beta = 1e-3
    scans = inputs.batch_scans(64)
    try:
        with open(os.path.join(GOLDEN, "batch64_census.json")) as fh:
            census = json.load(fh)
    except (OSError, ValueError):
        census = None
    torch.cuda.set_device(0)
    cache = autotune.load_cache(args.tune_cache) if args.tune_cache else {}
    geos, ys = [], []
    t_tune = time.perf_counter()
    for s in scans:
        f = torch.tensor(inputs.phantom(s.geom, s.phantom_seed, s.n_rect), dtype=torch.float32,
                         device="cuda")
        unit = csx.Geometry(s.geom.with_(C=1.0))
        l1 = unit.forward(f).double().cpu().numpy()
        unit.close()
        C = 1e4 / float(l1.max())
        geo = csx.Geometry(s.geom.with_(C=C))
        autotune.tuned(geo, cache)
        geos.append(geo)
        ys.append(torch.tensor(inputs.poisson_counts(C * l1, s.noise_seed), dtype=torch.float32,
                               device="cuda"))
    t_tune = time.perf_counter() - t_tune
    if args.tune_cache:
        autotune.save_cache(cache, args.tune_cache)
    batch = csx.Batch(geos)
    fb = [g.new_image() for g in geos]
    fs = [g.new_image() for g in geos]
    if args.warmup:
        batch.recon(ys, fb, args.warmup, beta)
        for g, y, f in zip(geos, ys, fs):
            g.recon(y, f, args.warmup, beta)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Jb = batch.recon(ys, fb, args.steps, beta)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    Js = [g.recon(y, f, args.steps, beta) for g, y, f in zip(geos, ys, fs)]
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    same = all(torch.equal(a, b) for a, b in zip(fb, fs)) and all(
        np.array_equal(Jb[k], Js[k]) for k in range(len(geos)))

    steps = max(1, args.steps)
    nominal = sum(2.0 * g.nvox * g.npix * g.nq for g in (s.geom for s in scans))
    ms_b = (t1 - t0) * 1e3 / steps
    ms_s = (t2 - t1) * 1e3 / steps
    roofline = None
    iv = [g.interval_operators()["on"] for g in geos]
    if all(iv):
        # every scan runs the interval-form operators: HBM-bound, algorithmic
        # bytes of one forward and one adjoint per scan
        nbytes = 0.0
        for g, s in zip(geos, scans):
            nb = interval_bytes(s.geom, bool(g.info()["symmetric_lr"]))
            nbytes += nb["forward"] + nb["adjoint"]
        achieved = nbytes / (ms_b * 1e-3)
        roofline = {"bound": "hbm", "kernel": "whole batched iteration (forward + adjoint + solver)",
                    "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                    "frac": achieved / PEAK_HBM, "traffic": None, "bytes_per_step": nbytes,
                    "bytes_model": "interval-form records, tables, images and detectors of every scan's "
                                   "forward and adjoint"}
    elif census is not None and not any(iv):
        ops = 2.0 * sum(algorithmic_ops(c) for c in census)
        achieved = ops / (ms_b * 1e-3)
        roofline = {"bound": "alu", "kernel": "whole batched iteration (forward + adjoint + solver)",
                    "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12, "unit": "TOP/s",
                    "frac": achieved / PEAK_LANE_OPS, "traffic": None, "ops_per_step": ops}
    sizes = {}
    for s in scans:
        key = f"{s.geom.nx}^2x{s.geom.nq}q"
        sizes[key] = sizes.get(key, 0) + 1
    out = {
        "metric": "fwd+adjoint voxel*pixel*energy evals/s, 64-scan uneven batch (one Alg. 5 iteration "
                  "of every scan per step)",
        "value": nominal / (ms_b * 1e-3), "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_b, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch64", "scans": len(scans), "sizes": sizes, "beta": beta,
                   "nominal_evals_per_step": nominal,
                   "timed": "csx_batch_recon of all scans (graph capture, uniform start and final "
                            "objective included) vs csx_recon per scan in turn"},
        "sequential": {"value": nominal / (ms_s * 1e-3), "ms_per_step": ms_s},
        "speedup_vs_sequential": ms_s / ms_b,
        "batched_equals_sequential": bool(same),
        "interval_scans": int(sum(iv)),
        "autotune_s": t_tune, "autotune_classes": len(cache),
        "roofline": roofline,
    }
    print(json.dumps(out))


def bench_paper(args):
    """The paper's simulation shape (Sec. VII): 28^2 voxels x 79 q, a 1536 x
    2048 detector of 0.19 mm pixels, stand-ins for the spectrum and mask, the
    two-vial phantom.  Beyond the interval form's limits, so the direct
    operators run, reading the factor store (22.8 GB, built at init); the
    adjoint splits its pixel classes into tile ranges.  A step is one Alg. 5
    iteration (Poisson counts around the phantom's forward, peak mean 1e4),
    timed with the autotuner's launch shape.  Context: the paper's Table 1
    times this shape's operators in MATLAB on a 12-core CPU."""
    import torch

    from paper_1603_06400_amd import csx, inputs

    torch.cuda.set_device(0)
    g0 = inputs.paper_geometry()
    unit = csx.Geometry(g0)
    ftrue = torch.tensor(inputs.paper_phantom(g0), dtype=torch.float32, device="cuda")
    mean = unit.forward(ftrue).double().cpu().numpy()
    unit.close()
    C = 1e4 / float(mean.max())
    g = g0.with_(C=C)
    geo = csx.Geometry(g)
    y = torch.tensor(inputs.poisson_counts(C * mean, 1), dtype=torch.float32, device="cuda")
    f = geo.new_image()
    geo.recon(y, f, max(1, args.warmup), 1e-3, init_uniform=True)

    def med(fn, n=10):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(n):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    gout, bout = geo.new_detector(), geo.new_image()
    fwd = med(lambda: geo.forward(f, gout))
    adj = med(lambda: geo.backproject(y, bout))
    lc = geo.get_launch()
    geo.set_launch(lc["fwd_splits"], lc["fwd_qw"], lc["adj_qw"], 1)
    adj1 = med(lambda: geo.backproject(y, bout))
    geo.set_launch(lc["fwd_splits"], lc["fwd_qw"], lc["adj_qw"], lc["adj_splits"])
    # the autotuner's shape (q chunk widths, forward voxel splits, adjoint class ranges)
    from paper_1603_06400_amd import autotune
    tuned = autotune.tune(geo, reps=3)
    fwd_t = med(lambda: geo.forward(f, gout))
    adj_t = med(lambda: geo.backproject(y, bout))
    J = torch.zeros(max(1, args.steps), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        geo.recon_step(y, f, 1e-3, J=J[k:k + 1])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / max(1, args.steps)
    trip = float(g.nvox) * g.npix * g.nq
    print(json.dumps({
        "metric": "fwd+adjoint voxel*pixel*energy evals/s, paper shape 28^2 x 79q x 1536x2048 (one Alg. 5 "
                  "iteration per step)",
        "value": 2.0 * trip / (ms * 1e-3), "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "paper_shape", "voxels": [g.nz, g.nx], "nq": g.nq, "detector": [g.ndy, g.ndx],
                   "ne": g.ne, "triples_per_operator": trip, "operators": "direct (beyond the interval form)",
                   "launch": geo.get_launch()},
        "factor_store": geo.factor_store(),
        "default_launch": {"forward_ms": fwd, "adjoint_ms": adj, "adjoint_ms_unsplit": adj1},
        "tuned_launch": {"shape": {k: tuned[k] for k in ("fwd_splits", "fwd_qw", "adj_qw", "adj_splits")},
                         "forward_ms": fwd_t, "adjoint_ms": adj_t},
        "objective_first_last": [float(J[0]), float(J[-1])] if args.steps else None,
        "context": {"paper_table1_matlab_12core_s": {"forward_no_opt": 10516.88, "backward_no_opt": 10512.32,
                                                      "forward_sai": 319.45, "backward_sai": 1191.05}},
    }))


def bench_os(args):
    """Ordered subsets (Alg. 6) with the paper's 64-subset partition on the
    128^2 x 64q slice and its stored counts: a step is one sweep over all
    subsets plus the full objective.  Nominal evals per sweep: one forward and
    one adjoint over all pixels (the subsets cover the detector once) plus the
    objective's forward."""
    import torch

    from paper_1603_06400_amd import csx, inputs

    phases = {}
    tp = time.perf_counter()
    w = inputs.workload(WORKLOAD)
    z = np.load(os.path.join(GOLDEN, f"{WORKLOAD}_counts.npz"))
    g = w.geom.with_(C=float(z["C"]))
    torch.cuda.set_device(0)
    geo = csx.Geometry(g)
    y = torch.tensor(z["y"], dtype=torch.float32, device="cuda")
    f = geo.new_image()
    geo.recon_os(y, f, max(1, args.warmup), w.beta, 8, 16)          # builds the partition
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = geo.recon_os(y, f, args.steps, w.beta, 8, 16, init_uniform=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / max(1, args.steps)
    nominal = 3.0 * g.nvox * g.npix * g.nq
    print(json.dumps({"metric": "ordered-subsets sweeps, 128^2 x 64q, 64 subsets (voxel*pixel*energy evals/s)",
                      "value": nominal / (ms * 1e-3), "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": "slice128_os64", "rho_z": 8, "rho_y": 16, "beta": w.beta,
                                 "nominal_evals_per_step": nominal},
                      "objective": [float(v) for v in J]}))


def bench_sai(args):
    """Scatter-angle interpolation (Sec. III-B) on the 128^2 x 64q slice: a
    step is one Alg. 5 iteration with both operators interpolated (N_theta =
    250, the paper's table size; linear nodes by default).  Also reported: the
    event-timed operators beside the exact ones, the operators' NRMSE against
    the exact ones (the paper's Table 1 measure: forward on the phantom,
    adjoint on its noiseless data) over table sizes and both node rules, and
    the reconstruction after 50 iterations against the exact operators'."""
    import torch

    from paper_1603_06400_amd import csx, inputs

    phases = {}
    tp = time.perf_counter()
    w = inputs.workload(WORKLOAD)
    z = np.load(os.path.join(GOLDEN, f"{WORKLOAD}_counts.npz"))
    g = w.geom.with_(C=float(z["C"]))
    torch.cuda.set_device(0)
    geo = csx.Geometry(g)
    f_true = torch.tensor(inputs.phantom(w.geom, w.phantom_seed, w.n_rect), dtype=torch.float32, device="cuda")
    y = torch.tensor(z["y"], dtype=torch.float32, device="cuda")

    def nrmse(a, b):
        return float(torch.linalg.norm((a - b).double()) / torch.linalg.norm(b.double()))

    g_ex = geo.forward(f_true)
    b_ex = geo.backproject(g_ex.clone())
    accuracy = []
    for interp in ("nearest", "linear"):
        for nt in (64, 250, 1000, 2000, csx.SAI_MAX_NODES):
            geo.sai_config(nt, interp)
            accuracy.append({"nt": nt, "interp": interp,
                             "forward_nrmse": nrmse(geo.forward_sai(f_true), g_ex),
                             "adjoint_nrmse": nrmse(geo.backproject_sai(g_ex), b_ex)})
    nt, interp = 250, args.sai_interp
    geo.sai_config(nt, interp)

    def timed(fn, n):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    gbuf, bbuf = geo.new_detector(), geo.new_image()
    ops = {"forward_sai_ms": timed(lambda: geo.forward_sai(f_true, gbuf), 20),
           "adjoint_sai_ms": timed(lambda: geo.backproject_sai(y, bbuf), 20),
           "forward_exact_ms": timed(lambda: geo.forward(f_true, gbuf), 20),
           "adjoint_exact_ms": timed(lambda: geo.backproject(y, bbuf), 20)}

    # Alg. 5 steps with both operators interpolated
    geo.set_operator(forward_sai=True, adjoint_sai=True)
    f_d = geo.new_image()
    J = torch.zeros(max(1, args.steps), dtype=torch.float64, device="cuda")
    geo.recon(y, f_d, 0, w.beta, init_uniform=True)
    for _ in range(args.warmup):
        geo.recon_step(y, f_d, w.beta, J=J[:1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        geo.recon_step(y, f_d, w.beta, J=J[k:k + 1])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / max(1, args.steps)
    # ordered subsets (Alg. 6, 64 subsets) on the interpolated operators, as the
    # paper runs its reconstructions, beside the exact operators' sweep
    def os_sweep_ms():
        fo = geo.new_image()
        geo.recon_os(y, fo, 1, w.beta, 8, 16)            # builds the partition and sensitivities
        torch.cuda.synchronize()
        t = time.perf_counter()
        J_os = geo.recon_os(y, fo, 3, w.beta, 8, 16, init_uniform=True)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / 3, J_os
    os_sai_ms, J_os_sai = os_sweep_ms()
    # reconstructions: 50 iterations with interpolated and with exact operators
    f_sai = geo.new_image()
    geo.recon(y, f_sai, w.n_iter, w.beta)
    geo.set_operator()
    os_exact_ms, J_os_exact = os_sweep_ms()
    f_ex = geo.new_image()
    J_ex = geo.recon(y, f_ex, w.n_iter, w.beta)
    t2 = time.perf_counter()
    geo.recon(y, f_ex, w.n_iter, w.beta)
    torch.cuda.synchronize()
    ms_exact_step = (time.perf_counter() - t2) * 1e3 / w.n_iter
    nominal = 2.0 * g.nvox * g.npix * g.nq
    print(json.dumps({
        "metric": "fwd+adjoint voxel*pixel*energy evals/s at 128^2 x 64q, Alg. 5 with interpolated scatter "
                  "angles (N_theta = 250; nominal evals counted as if exact)",
        "value": nominal / (ms * 1e-3), "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "slice128_sai", "nt": nt, "interp": interp, "theta_max": geo.sai_info()["theta_max"],
                   "beta": w.beta, "nominal_evals_per_step": nominal},
        "operators": ops, "ms_per_exact_step": ms_exact_step, "speedup_step": ms_exact_step / ms,
        "os64_sweep_ms": {"interpolated": os_sai_ms, "exact": os_exact_ms},
        "os64_objective_3_sweeps": {"interpolated": [float(v) for v in J_os_sai],
                                    "exact": [float(v) for v in J_os_exact]},
        "accuracy": accuracy,
        "recon_nrmse_vs_exact": nrmse(f_sai, f_ex), "n_iter": w.n_iter,
        "objective_exact_last": float(J_ex[-1])}))


def bench_energy(args):
    """The energy-sensitive detector (App. A) on the 128^2 x 64q slice with a
    64-bin energy-resolving detector: a step is one Alg. 5 iteration on the
    [64][128][128] counts (forward, ratio, adjoint, update, objective).  The
    counts are Poisson draws around the library's own energy-resolved forward
    of the workload phantom (seeded).  Also reported: the event-timed energy
    operators beside the energy-integrating ones."""
    import torch

    from paper_1603_06400_amd import csx, inputs

    phases = {}
    tp = time.perf_counter()
    w = inputs.workload(WORKLOAD)
    z = np.load(os.path.join(GOLDEN, f"{WORKLOAD}_counts.npz"))
    g = w.geom.with_(C=float(z["C"]))
    torch.cuda.set_device(0)
    geo = csx.Geometry(g)
    f_true = torch.tensor(inputs.phantom(w.geom, w.phantom_seed, w.n_rect), dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(7)
    yE = torch.poisson(geo.forward_energy(f_true).clamp_min(0.0), generator=gen)
    y = torch.tensor(z["y"], dtype=torch.float32, device="cuda")

    def timed(fn, n):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    gE, b, gbuf = torch.empty_like(yE), geo.new_image(), geo.new_detector()
    ops = {"forward_energy_ms": timed(lambda: geo.forward_energy(f_true, gE), 10),
           "adjoint_energy_ms": timed(lambda: geo.backproject_energy(yE, b), 10),
           "forward_exact_ms": timed(lambda: geo.forward(f_true, gbuf), 10),
           "adjoint_exact_ms": timed(lambda: geo.backproject(y, b), 10)}
    f = geo.new_image()
    geo.recon_energy(yE, f, max(1, args.warmup), w.beta)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = geo.recon_energy(yE, f, args.steps, w.beta)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / max(1, args.steps)
    nominal = 2.0 * g.nvox * g.npix * g.nq
    print(json.dumps({
        "metric": "fwd+adjoint voxel*pixel*energy evals/s at 128^2 x 64q, Alg. 5 on energy-resolved counts "
                  "(64 energy bins per pixel)",
        "value": nominal / (ms * 1e-3), "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic (Poisson around the library's forward)",
        "config": {"workload": "slice128_energy", "ne": g.ne, "beta": w.beta, "nominal_evals_per_step": nominal},
        "operators": ops, "objective": [float(J[0]), float(J[-1])]}))


def time_to_objective(n_cases: int, batched: bool = False, log=None) -> dict:
    """Time for the plain solver, for the judged learned warm start (network
    and judge included) and for ordered subsets (Alg. 6, 64 subsets) to reach
    J_plain(50) (1 + 1e-3) on held-out phantoms of the 128^2 x 64q slice;
    with batched, the warm path also runs batched over the cases."""
    from paper_1603_06400_amd import csx, inputs, warmstart
    w, g = warmstart.calibrated_geometry()
    net = warmstart.WarmNet.load()
    cases = inputs.warm_cases("eval", n_cases)
    geo = csx.Geometry(g)
    # the partition's lists and sensitivities are built once per handle
    geo.recon_os(geo.new_detector().fill_(1.0), geo.new_image(), 0, w.beta, 8, 16)
    rows = warmstart.evaluate(geo, net, cases, w.n_iter, w.beta, k_judge=2, log=log, os_partition=(8, 16))
    out = warmstart.summarize(rows)
    out["target"] = "J <= J_plain(50) (1 + 1e-3), held-out phantoms"
    if batched:
        out["batched"] = warmstart.evaluate_batched(g, net, cases, w.n_iter, w.beta, k_judge=2, log=log)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the median operator launches and the 32^2 slice run (profiling runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (10 times), the "
                         "reference kernel for scaling HBM byte counters")
    ap.add_argument("--workload", default=WORKLOAD, choices=[WORKLOAD, "batch64", "warm", "os", "sai", "energy", "paper"],
                    help="slice128 (default): the single 128^2 x 64q slice; batch64: the batched form; "
                         "warm: time to the plain objective with the learned warm start; os: sweeps of "
                         "ordered subsets (Alg. 6, 64 subsets) on the slice; sai: Alg. 5 with "
                         "scatter-angle interpolation; energy: Alg. 5 on energy-resolved counts; paper: the paper's "
                         "28^2 x 79q x 1536x2048 shape (direct operators)")
    ap.add_argument("--sai-interp", default="linear", choices=["linear", "nearest"],
                    help="sai: node rule of the timed table")
    ap.add_argument("--tto-cases", type=int, default=4,
                    help="held-out phantoms for the time-to-objective entry (0: skip; warm workload: 200)")
    ap.add_argument("--tune-cache", default=None, metavar="PATH",
                    help="batch64: launch-shape cache file to read and update")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.rand(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 4 * n, "bytes_written": 4 * n, "launches": 10}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(independent scans shard across GPUs without communication).", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch64":
        bench_batch(args)
        return
    if args.workload == "os":
        bench_os(args)
        return
    if args.workload == "paper":
        bench_paper(args)
        return
    if args.workload == "sai":
        bench_sai(args)
        return
    if args.workload == "energy":
        bench_energy(args)
        return
    if args.workload == "warm":
        import torch
        torch.cuda.set_device(0)
        n = args.tto_cases if args.tto_cases != 4 else 200
        # the batched part runs in the default line (4 scans); over 200 cases
        # its 25-scan batches ended the process (cause not found; the batch
        # then ran its scans on parallel graph branches), so it is off
        tto = time_to_objective(n, batched=False, log=lambda m: print(m, file=sys.stderr, flush=True))
        tto["batched"] = "off for this workload: 25-scan batches ended the process with a segmentation fault"
        print(json.dumps({"metric": "time to the plain solver's objective (1e-3 relative), 128^2 x 64q slice",
                          "value": tto["speedup_mean_time"], "unit": "x (plain time / warm time)",
                          "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
                          "config": {"workload": "warm", "cases": n}, "time_to_objective": tto}))
        return

    import torch

    from paper_1603_06400_amd import csx, inputs

    phases = {}
    tp = time.perf_counter()
    w = inputs.workload(WORKLOAD)
    z = np.load(os.path.join(GOLDEN, f"{WORKLOAD}_counts.npz"))
    g = w.geom.with_(C=float(z["C"]))
    y = z["y"].astype(np.float64)
    with open(os.path.join(GOLDEN, f"{WORKLOAD}_census.json")) as fh:
        census = json.load(fh)
    torch.cuda.set_device(0)
    geo = csx.Geometry(g)
    ivi = geo.interval_operators()
    y_d = torch.tensor(y, dtype=torch.float32, device="cuda")
    f_d = geo.new_image()
    J = torch.zeros(max(1, args.steps), dtype=torch.float64, device="cuda")

    # f^0 and the sensitivity image (uniform start, zero iterations)
    geo.recon(y_d, f_d, 0, w.beta, init_uniform=True)
    for _ in range(args.warmup):
        geo.recon_step(y_d, f_d, w.beta, J=J[:1])
    torch.cuda.synchronize()

    geo.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        geo.recon_step(y_d, f_d, w.beta, J=J[k:k + 1])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tim = geo.timing_read()
    geo.timing_enable(False)

    ms_step = (t1 - t0) * 1e3 / max(1, args.steps)
    nominal = 2.0 * g.nvox * g.npix * g.nq
    value = nominal / (ms_step * 1e-3)
    Jh = J.cpu().numpy()

    fwd_ms = tim["forward_ms"] / max(1, tim["forward_n"])
    adj_ms = tim["adjoint_ms"] / max(1, tim["adjoint_n"])
    phases["gpu_setup_and_timed_steps_s"] = time.perf_counter() - tp
    store = geo.factor_store()
    lr = bool(geo.info()["symmetric_lr"])
    dom = "adjoint" if adj_ms >= fwd_ms else "forward"
    dom_ms = max(adj_ms, fwd_ms)
    if ivi["on"]:
        nb = interval_bytes(g, lr)
        kname = "k_iv_adjoint" if dom == "adjoint" else "k_iv_forward"
        achieved = nb[dom] / (dom_ms * 1e-3)
        traffic = stored_traffic(kname)
        roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9,
                    "unit": "GB/s", "frac": achieved / PEAK_HBM, "traffic": traffic,
                    "bytes_per_launch": nb[dom], "bytes_model": "8 B per class record (forward: slot order; adjoint: interval order) + the "
                    "adjoint's 2 B table index per (node, bin edge) and 1 B position mask per 8 ranks, per "
                    "voxel group + image + detector arrays",
                    "forward_ms": fwd_ms, "adjoint_ms": adj_ms,
                    "forward_GB_per_s": nb["forward"] / (fwd_ms * 1e-3) / 1e9,
                    "adjoint_GB_per_s": nb["adjoint"] / (adj_ms * 1e-3) / 1e9}
    else:
        ops = algorithmic_ops(census, stored=store["on"], pairs_per_class=4 if lr else 2)
        kname = "k_adjoint" if dom == "adjoint" else "k_forward"
        achieved = ops / (dom_ms * 1e-3)
        measured_peak = csx.valu_peak()
        traffic = stored_traffic(kname)
        roofline = {"bound": "alu", "kernel": dom, "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                    "unit": "TOP/s", "frac": achieved / PEAK_LANE_OPS, "traffic": traffic,
                    "traffic_GB_per_s": None if traffic is None else traffic / (dom_ms * 1e-3) / 1e9,
                    "ops_per_launch": ops,
                    "op_model": ("4 per open in-band triple + 20 per stored class record" if store["on"] else
                                 "4 per open in-band triple + 60 per open pair + 10 per pair"),
                    "forward_ms": fwd_ms, "adjoint_ms": adj_ms,
                    "peak_measured": measured_peak / 1e12, "frac_of_measured": achieved / measured_peak}

    out = {
        "metric": "fwd+adjoint voxel*pixel*energy evals/s at 128^2 x 64q (one Alg. 5 iteration per step)",
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD, "voxels": [g.nz, g.nx], "nq": g.nq, "detector": [g.ndy, g.ndx],
                   "ne": g.ne, "mask_open": float(g.mask.mean()), "beta": w.beta,
                   "nominal_evals_per_step": nominal},
        "roofline": roofline,
        "operators": {"interval_form": ivi, "class_store": store},
        "objective_first_last": [float(Jh[0]), float(Jh[-1])] if args.steps else None,
    }
    if not args.no_extras:
        tp = time.perf_counter()
        out["operator_median"] = operator_medians(geo, f_d, y_d)
        out["slice32_gpu"] = gpu_slice32()
        phases["operator_medians_and_slice32_s"] = time.perf_counter() - tp
    if args.tto_cases > 0:
        tp = time.perf_counter()
        tto = time_to_objective(args.tto_cases, batched=True)
        out["time_to_objective"] = {k: tto[k] for k in ("cases", "target", "ms_plain_mean", "ms_warm_mean",
                                                         "speedup_mean_time", "iters_plain_mean",
                                                         "iters_warm_mean", "accept_rate", "ms_os_mean",
                                                         "os_sweeps_mean", "speedup_os_mean_time", "batched")}
        phases["time_to_objective_s"] = time.perf_counter() - tp
    if not args.no_cpu_baseline:
        tp = time.perf_counter()
        f_true = inputs.phantom(w.geom, w.phantom_seed, w.n_rect)
        out["cpu_baseline"] = cpu_baseline(g, f_true, y)
        phases["cpu_baseline_s"] = time.perf_counter() - tp
    out["phases_wall_s"] = phases
    print(json.dumps(out))


if __name__ == "__main__":
    main()
