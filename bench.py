#!/usr/bin/env python
"""Benchmark of the batched robust shifted-Hessenberg solve on one MI355X.

Workload (the configuration the headline metric is quoted on): n = 8000,
m = 1000 real shifts, the random unreduced Hessenberg matrix of the n = 2000
configuration (entries N(0,1) on and above the diagonal, subdiagonal
|N(0,1)| + 0.1, seed 1003) graded by D H D^-1 with D_ii = 10^(300 i / n);
shifts are real eigenvalues of the ungraded matrix computed on the host;
starting vectors all ones.  One step = one complete solve of the 1000 shifts
(every kernel of the path), with H, shifts and starting vectors already
resident in device memory.  The headline times K solves replayed from the
library's captured HIP graph; the same K solves are then run kernel by kernel
twice: plain, and with HIP timing events attached to every step-kernel
dispatch (hipExtLaunchKernelGGL, on the stream of each launch), which cost a
few per cent of wall time and therefore stay out of the headline pass.

Prints one JSON line.  ``roofline`` is for the kernel family with the
largest measured time per solve (the critical kernel: superdiagonal tile and
diagonal chain, or the far-tile kernel: off-diagonal tile updates and
rotations), from the durations of the event pass; ``kernels`` gives both.  ``traffic`` (HBM bytes per
launch) comes from rocprofv3 FETCH_SIZE / WRITE_SIZE counter runs committed
under profiles/, calibrated against a plain device copy (``--copy-probe``),
and is null when the kernel sources changed since they were taken.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6       # MI355X FP64 vector and FP64 matrix (dense)
PEAK_HBM_GBS = 8000.0


def table1_flops(n, nb, wi):
    """Algorithmic flops of one solve after Table 1 of the paper, summed over
    the tile grid (tiles aligned to the bottom-right, ragged top-left tile):
    per real column ReduceDiag 1.5 h^2 and Solve 3.5 h^2 per diagonal tile of
    order h, ReduceOffdiag 3 r b and Update 2 r b per off-diagonal tile of r
    rows and b columns, back-transform 6 (n - 1); per complex vector (two
    columns) 3 h^2, 15 h^2, 6 r b, 4 r b and 20 (n - 1).
    Returns a dict: far (off-diagonal tiles not adjacent to the diagonal:
    the far-tile kernel), crit (superdiagonal tiles + diagonal tiles: the
    critical kernel), update (the level-3 part: Update of every
    off-diagonal tile), far_update (the Update of the tiles in the far-tile
    kernel), total."""
    import numpy as np
    N = (n + nb - 1) // nb
    ends = [n - (N - 1 - t) * nb for t in range(N)]
    starts = [max(0, e - nb) for e in ends]
    sizes = [e - s for s, e in zip(starts, ends)]
    diag2 = sum(h * h for h in sizes)
    # off-diagonal tile (i, jt), i < jt: rows sizes[i], width nb
    super_rows = sum(sizes[jt - 1] for jt in range(1, N))
    far_rows = sum(sum(sizes[:jt - 1]) for jt in range(2, N))
    nreal = int(np.sum(np.asarray(wi) == 0))
    ncplx = len(wi) - nreal
    per_r, per_c = 5.0, 10.0          # ReduceOffdiag + Update per row and tile column
    diag_r, diag_c = 5.0, 18.0        # ReduceDiag + Solve per h^2
    far = nb * far_rows * (per_r * nreal + per_c * ncplx)
    crit = nb * super_rows * (per_r * nreal + per_c * ncplx) + diag2 * (diag_r * nreal + diag_c * ncplx)
    update = nb * (far_rows + super_rows) * (2.0 * nreal + 4.0 * ncplx)
    far_update = nb * far_rows * (2.0 * nreal + 4.0 * ncplx)
    back = 6.0 * (n - 1) * nreal + 20.0 * (n - 1) * ncplx
    return dict(far=far, crit=crit, update=update, far_update=far_update, total=far + crit + back)


def kernel_source_hash():
    """Hash of the device-code sources (the kernels and the layout header
    they share): counter figures are valid only for the kernels they were
    taken on."""
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2101_05063_amd", "csrc")
    for f in ("hsrq_kernels.hip", "hsrq_common.h"):
        h.update(open(os.path.join(src, f), "rb").read())
    return h.hexdigest()[:16]


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_c3.json")


def load_traffic(kernel):
    """HBM bytes per launch of `kernel` (a name, or names joined by " + " for a
    family launched as several kernels: launch-weighted) from the committed
    counter runs, valid only for the kernel sources they were taken on."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    d = json.load(open(TRAFFIC_FILE))
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    ks = [d.get("kernels", {}).get(name) for name in kernel.split(" + ")]
    if any(k is None for k in ks):
        return None
    launches = sum(k["launches"] for k in ks)
    return sum(k["bytes_per_launch"] * k["launches"] for k in ks) / launches if launches else None


def _pmc_rows(path):
    """(kernel name, counter value) rows of a rocprofv3 counter_collection.csv."""
    import csv
    out = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            out.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return out


def ingest_pmc(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes):
    """Writes profiles/traffic_c3.json from two counter runs of the benchmark
    (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch) and the same two counters
    read on the plain copy of --copy-probe, whose true traffic is copy_bytes
    read and copy_bytes written per dispatch."""
    import statistics

    def per_kernel(rows):
        acc = {}
        for name, v in rows:
            key = name.split("(")[0].replace("void ", "").strip()
            acc.setdefault(key, []).append(v)
        return acc

    def copy_value(rows):
        vals = [v for name, v in rows if "copy" in name.lower()]
        return statistics.median(vals)

    f_copy = copy_value(_pmc_rows(copy_fetch_csv)) * 1024.0
    w_copy = copy_value(_pmc_rows(copy_write_csv)) * 1024.0
    f_scale, w_scale = copy_bytes / f_copy, copy_bytes / w_copy
    fk, wk = per_kernel(_pmc_rows(fetch_csv)), per_kernel(_pmc_rows(write_csv))
    kernels = {}
    for k in fk:
        if k in wk:
            fb = statistics.mean(fk[k]) * 1024.0 * f_scale
            wb = statistics.mean(wk[k]) * 1024.0 * w_scale
            kernels[k] = {"fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                          "bytes_per_launch": fb + wb, "launches": len(fk[k])}
    d = {"kernel_source_hash": kernel_source_hash(), "copy_bytes": copy_bytes,
         "fetch_scale": f_scale, "write_scale": w_scale, "kernels": kernels}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    print(json.dumps(d, indent=1, sort_keys=True))


MFMA_FILE = os.path.join(ROOT, "profiles", "mfma_c3.json")


def ingest_mfma(pmc_csv, stats_csv):
    """Writes profiles/mfma_c3.json from a rocprofv3 counter run of the
    benchmark (SQ_VALU_MFMA_BUSY_CYCLES, SQ_INSTS_VALU_MFMA_MOPS_F64,
    SQ_WAIT_INST_ANY, SQ_WAVE_CYCLES) and the kernel statistics of a
    kernel-trace run of the same command: per kernel the MFMA flops per
    launch (MOPS_F64 counts units of 512 flops) and the fraction of the
    1024 SIMDs' cycles over the average launch duration that the matrix
    cores were busy."""
    import csv
    import statistics
    acc = {}
    with open(pmc_csv, newline="") as f:
        for r in csv.DictReader(f):
            key = r["Kernel_Name"].split("(")[0].replace("void ", "").strip()
            d = acc.setdefault(key, {}).setdefault(r["Counter_Name"], {})
            d.setdefault(r.get("Dispatch_Id", str(len(d))), 0.0)
            d[r.get("Dispatch_Id", str(len(d)))] += float(r["Counter_Value"])
    avg_ns = {}
    with open(stats_csv, newline="") as f:
        for r in csv.DictReader(f):
            avg_ns[r["Name"].split("(")[0].replace("void ", "").strip()] = float(r["AverageNs"])
    kernels = {}
    for k, cs in acc.items():
        if k not in avg_ns or "SQ_VALU_MFMA_BUSY_CYCLES" not in cs:
            continue
        mean = {c: statistics.mean(v.values()) for c, v in cs.items()}
        busy = mean["SQ_VALU_MFMA_BUSY_CYCLES"] / (1024 * 2.4e9 * avg_ns[k] * 1e-9)
        ent = {"avg_launch_us": avg_ns[k] / 1e3, "mfma_busy": round(busy, 4),
               "dispatches": len(next(iter(cs.values())))}
        if "SQ_INSTS_VALU_MFMA_MOPS_F64" in mean:
            ent["mfma_flops_per_launch"] = mean["SQ_INSTS_VALU_MFMA_MOPS_F64"] * 512.0
        if "SQ_WAIT_INST_ANY" in mean and "SQ_WAVE_CYCLES" in mean and mean["SQ_WAVE_CYCLES"] > 0:
            ent["wave_cycles_waiting"] = round(mean["SQ_WAIT_INST_ANY"] / mean["SQ_WAVE_CYCLES"], 4)
        kernels[k] = ent
    d = {"kernel_source_hash": kernel_source_hash(), "kernels": kernels}
    with open(MFMA_FILE, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    print(json.dumps(d, indent=1, sort_keys=True))


COPY_BYTES = 256 << 20


def copy_probe():
    """A plain device copy of known size for calibrating the HBM counters."""
    import torch
    n = COPY_BYTES // 8
    a = torch.rand(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": COPY_BYTES, "dispatches": 5}), flush=True)


def cpu_model():
    """The host CPU's model name (as lscpu reports it), from /proc/cpuinfo."""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_reference_c3(c, seconds, cores):
    """The plain C reference on the C3 shifts, on `cores` threads: all of them
    when that is expected to take at most `seconds`, else a stratified subset
    (every k-th shift of the list, so that the sample spans the whole range of
    eigenvalues and exponents).  The expectation comes from a probe of
    `cores` shifts spread over the list.  Returns (cpu_baseline dict, sample
    indices, reference outputs on the sample)."""
    import numpy as np

    from oracle import oracle as O
    H, wr, wi, B = c["H"], c["wr"], c["wi"], c["B"]
    m = len(wr)
    O.build()
    probe = np.linspace(0, m - 1, max(1, cores)).round().astype(int)
    t0 = time.perf_counter()
    O.batch(H, wr[probe], wi[probe], B[:, probe], nthreads=cores)
    per_shift = max(time.perf_counter() - t0, 1e-3) / len(probe)
    k = max(1, int(np.ceil(m * per_shift / seconds)))
    sel = np.arange(0, m, k)
    t0 = time.perf_counter()
    Yo, Eo, muo, infoo = O.batch(H, wr[sel], wi[sel], B[:, sel], nthreads=cores)
    dt = time.perf_counter() - t0
    base = dict(value=len(sel) / dt, unit="eigenvectors/s", cores=cores, kind="oracle", cpu_model=cpu_model(),
                sample=(f"all {m} shifts of the C3 workload (n={H.shape[0]})" if k == 1 else
                        f"{len(sel)} of the {m} C3 shifts (one in {k}, n={H.shape[0]})") +
                       f", {dt:.1f} s wall on {cores} threads")
    return base, sel, (Yo, Eo, muo, infoo)


def error_vs_reference_c3(Yg, Eg, mug, infog, sel, ref, wi):
    """Per-result error of one C3 solve against the reference on the sampled
    shifts: flags, exponents (binade straddles within 1e-6 in log2 reported
    apart), mantissas, directions."""
    import numpy as np
    Yo, Eo, muo, infoo = ref
    Eg, mug, infog = Eg[sel], mug[sel], infog[sel]
    Yg = Yg[:, sel]
    d = np.abs(np.sum(Yg * Yo, axis=0)) / (np.linalg.norm(Yg, axis=0) * np.linalg.norm(Yo, axis=0))
    same = Eg == Eo
    lg = Eo + np.log2(np.where(muo > 0, muo, 1.0))
    straddle = (~same) & (np.abs(Eg - Eo) == 1) & (np.abs(lg - np.round(lg)) < 1e-6)
    rel = np.abs(mug[same] - muo[same]) / muo[same]
    return {"results": int(len(sel)), "flag_mismatches": int(np.sum(infog != infoo)),
            "exponent_mismatches": int(np.sum(~same & ~straddle)),
            "exponent_binade_straddles": int(np.sum(straddle)),
            "max_rel_mantissa_diff": float(rel.max()) if rel.size else 0.0,
            "median_rel_mantissa_diff": float(np.median(rel)) if rel.size else 0.0,
            "max_1_minus_cos": float(max(0.0, (1.0 - d).max()))}


def error_vs_reference(probs_h, probs_d, outs, cores):
    """Per-result error of a GPU solve against the plain CPU reference (every
    shift of every problem): 1 - |cos| of the directions, exponent mismatches
    (binade straddles excepted), relative mantissa difference."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as O
    O.build()

    def one(b):
        pr = probs_h[b]
        return O.batch(pr["H"], pr["wr"], pr["wi"], pr["B"], nthreads=1)

    with ThreadPoolExecutor(max_workers=cores) as ex:
        refs = list(ex.map(one, range(len(probs_h))))
    dir_err, mu_err, e_mis, straddle = [], [], 0, 0
    for pr, pd, (E, mu, info, _), (Yo, Eo, muo, infoo) in zip(probs_h, probs_d, outs, refs):
        Yg = pd["X"].t().contiguous().cpu().numpy().T
        E, mu = E.cpu().numpy(), mu.cpu().numpy()
        cols, _ = O.columns_of(pr["wi"])
        for l in range(len(pr["wr"])):
            c = cols[l]
            if pr["wi"][l] != 0.0:
                yg = Yg[:, c] + 1j * Yg[:, c + 1]
                yo = Yo[:, c] + 1j * Yo[:, c + 1]
            else:
                yg, yo = Yg[:, c], Yo[:, c]
            d = abs(np.vdot(yg, yo)) / (np.linalg.norm(yg) * np.linalg.norm(yo))
            dir_err.append(max(0.0, 1.0 - d))
            if E[l] != Eo[l]:
                lg = Eo[l] + np.log2(muo[l])
                if abs(E[l] - Eo[l]) == 1 and abs(lg - round(lg)) < 1e-4:
                    straddle += 1
                else:
                    e_mis += 1
            else:
                mu_err.append(abs(mu[l] - muo[l]) / muo[l])
    dir_err = np.array(dir_err)
    return {"results": int(dir_err.size), "max_1_minus_cos": float(dir_err.max()),
            "p99_1_minus_cos": float(np.quantile(dir_err, 0.99)),
            "max_rel_mantissa_diff": float(max(mu_err) if mu_err else 0.0),
            "exponent_mismatches": e_mis, "exponent_binade_straddles": straddle}


def bench_c4(args):
    """Batching: the 512 matrices of uneven order (n log-uniform in
    [64, 2048], 4-64 shifts each, 30% complex pairs) solved together, the
    tile size chosen by the library's autotuner, each solve one replay of the
    captured launch sequence (precision 0).  With --precision 1 the
    mixed-precision solve (FP32 tile products, FP64 residual check, FP64
    fallback; not graph-replayed because of its host check) is timed, and
    every result's error against the CPU reference is reported.  One step =
    one solve of all 512 problems."""
    import numpy as np
    import torch

    from paper_2101_05063_amd import Solver
    from workloads import generators as g

    probs_h = g.config_c4()
    dev = torch.device("cuda:0")

    def todev(A):
        return torch.from_numpy(np.ascontiguousarray(np.asarray(A, dtype=np.float64).T)).to(dev).t()

    Hs = [todev(p["H"]) for p in probs_h]
    Bs = [todev(p["B"]) for p in probs_h]
    ncols = sum(B.shape[1] for B in Bs)
    nshift = sum(len(p["wr"]) for p in probs_h)
    solver = Solver(0)

    def problems():
        return [dict(H=H, wr=p["wr"], wi=p["wi"], X=B.clone()) for H, B, p in zip(Hs, Bs, probs_h)]

    best, best_cb, tune_ms = solver.autotune(problems(), precision=args.precision, rotations=args.rotations)

    def timed(graph):
        # every step solves its own copy of the starting vectors (the solve
        # overwrites X); the sets are marshalled before the timed region
        sets = [problems() for _ in range(args.warmup + args.steps)]
        preps = [solver.prepare(s) for s in sets]
        torch.cuda.synchronize()
        for k in range(args.warmup):
            solver.batched(preps[k], precision=args.precision, graph=graph, rotations=args.rotations)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = None
        for k in range(args.steps):
            outs = solver.batched(preps[args.warmup + k], precision=args.precision, graph=graph,
                                  rotations=args.rotations)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps, sets[-1], outs

    ms, last_set, outs = timed(1)
    fallback = solver.fallback_count() if args.precision == 1 else 0
    conv = float(np.mean(np.concatenate([o[2].cpu().numpy() == 0 for o in outs])))
    ms_eager, _, _ = timed(-1)
    line = {
        "metric": "eigenvectors/s (batching: 512 matrices of uneven order)",
        "value": round(ncols / (ms * 1e-3), 2), "unit": "eigenvectors/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == 0 else "f64+f32", "data": "synthetic",
        "config": {"workload": "512 random unreduced Hessenberg matrices, n log-uniform in [64, 2048], "
                               "4-64 host-eigenvalue shifts each (30% complex pairs), all-ones starts",
                   "matrices": len(probs_h), "sum_n": int(sum(p["H"].shape[0] for p in probs_h)),
                   "shifts": nshift, "columns": ncols, "precision": args.precision,
                   "rotations": args.rotations,
                   "autotuned_nb": best, "autotuned_cols_per_block": best_cb,
                   "autotune_ms": {f"nb={nb},cols_per_block={cb}": round(v, 4) for (nb, cb), v in tune_ms.items()},
                   "graph": args.precision == 0},
        "shifts_per_s": round(nshift / (ms * 1e-3), 2),
        "ms_per_step_kernel_by_kernel": round(ms_eager, 4),
        "converged_fraction": conv,
    }
    if args.precision == 1:
        line["fallback_shifts"] = fallback
    if args.precision == 1 or args.rotations == 1:
        line["error_vs_reference"] = error_vs_reference(probs_h, last_set, outs, len(os.sched_getaffinity(0)))
    solver.close()
    print(json.dumps(line), flush=True)


def bench_hessenberg(args):
    """The steps around the solve: Householder reduction of a general n x n
    matrix to Hessenberg form (hsrq_gehrd) and the back-transform of ncols
    vectors (hsrq_ormhr), on seeded standard-normal data.  One step = one
    reduction plus one back-transform.  The reduction is HBM-bound: its
    algorithmic bytes are one read and one write of the trailing matrix per
    reflector (16 n (n - q - 2) for reflector q).  The back-transform is
    blocked (compact WY) and runs as matrix products: its algorithmic flops
    are those of applying each reflector to the columns, 4 (n - q - 1) ncols
    for reflector q."""
    import numpy as np
    import torch

    from paper_2101_05063_amd import Solver

    n, ncols = args.hess_n, args.hess_cols
    rng = np.random.default_rng(2101)
    dev = torch.device("cuda:0")
    A0 = torch.from_numpy(np.ascontiguousarray(rng.standard_normal((n, n)).T)).to(dev).t()
    Z0 = torch.from_numpy(np.ascontiguousarray(rng.standard_normal((n, ncols)).T)).to(dev).t()
    solver = Solver(0)
    K, W = args.steps, args.warmup
    As = [A0.clone() for _ in range(K + W)]
    Zs = [Z0.clone() for _ in range(K + W)]
    torch.cuda.synchronize()
    taus = [solver.gehrd(As[k]) for k in range(W)]
    for k in range(W):
        solver.ormhr(As[k], taus[k], Zs[k])
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    t_red = t_bt = 0.0
    for k in range(W, W + K):
        e0.record()
        tau = solver.gehrd(As[k])
        e1.record()
        solver.ormhr(As[k], tau, Zs[k])
        e2.record()
        torch.cuda.synchronize()
        t_red += e0.elapsed_time(e1)
        t_bt += e1.elapsed_time(e2)
    ms_red, ms_bt = t_red / K, t_bt / K
    bytes_red = sum(16.0 * n * (n - q - 2) for q in range(n - 2))
    flops_bt = sum(4.0 * (n - q - 1) * ncols for q in range(n - 2))
    gbs_red = bytes_red / (ms_red * 1e-3) / 1e9
    tf_bt = flops_bt / (ms_bt * 1e-3) / 1e12
    # spot check of the last reduction: Q0 orthogonal on a few columns (Q0 e_j
    # from the back-transform of unit vectors)
    E = torch.zeros(n, 4, dtype=torch.float64, device=dev)
    idx = [0, n // 3, n // 2, n - 1]
    for j, i in enumerate(idx):
        E[i, j] = 1.0
    Q = solver.ormhr(As[-1], tau, E.t().contiguous().t())
    orth = float((Q.t() @ Q - torch.eye(4, dtype=torch.float64, device=dev)).abs().max())
    line = {
        "metric": "Hessenberg reduction + back-transform time (n x n general matrix, ncols vectors)",
        "value": round(ms_red + ms_bt, 3), "unit": "ms", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(ms_red + ms_bt, 3), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"general standard-normal matrix n={n}, back-transform of {ncols} vectors",
                   "n": n, "ncols": ncols},
        "reduction": {"ms": round(ms_red, 3), "algorithmic_bytes": bytes_red, "achieved_GBps": round(gbs_red, 1),
                      "frac_hbm_peak": round(gbs_red / PEAK_HBM_GBS, 4)},
        "back_transform": {"ms": round(ms_bt, 3), "algorithmic_flops": flops_bt,
                           "achieved_TFLOPs": round(tf_bt, 2), "frac_fp64_peak": round(tf_bt / PEAK_FP64_TFLOPS, 4)},
        "roofline": {"kernel": "hsrq::k_sweep (reduction, whole call)", "bound": "hbm",
                     "achieved": round(gbs_red, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(gbs_red / PEAK_HBM_GBS, 4), "traffic": None},
        "check": {"q0_orthogonality_4_columns": orth},
    }
    solver.close()
    print(json.dumps(line), flush=True)


def order_stat(x, q):
    """Exact order statistic: the smallest value with at least a fraction q of
    the sample at or below it."""
    import math
    xs = sorted(x)
    return xs[max(0, math.ceil(q * len(xs)) - 1)]


def serving_run(args, requests, warm):
    """Serving: requests on a pool of 64 random unreduced Hessenberg matrices
    (n log-uniform in [128, 8192]), each with U{1..n/8} host-eigenvalue shifts
    (30% complex pairs) and all-ones starts, H resident on the device.  First
    the saturated throughput is measured closed-loop (`warm` requests
    submitted at once after a warm-up of 20); then `requests` arrivals follow
    a Poisson process at 0.7 times that rate, submitted to the library's
    serving loop (HBM budget 200 GB) as they arrive.  Latency = completion -
    arrival on the server's clock; p50/p99 are exact order statistics."""
    import numpy as np
    import torch

    from paper_2101_05063_amd import Server
    from workloads import generators as g

    pool = g.config_c5_pool()
    dev = torch.device("cuda:0")
    Hd = [torch.from_numpy(np.ascontiguousarray(p["H"].T)).to(dev).t() for p in pool]
    rng = np.random.default_rng(1006)
    reqs = [(b, wr, wi, g.ncols(wi)) for b, wr, wi in g.c5_requests(pool, requests + warm)]
    srv = Server(0, budget_bytes=200 * 10 ** 9, nb=args.nb or 128, precision=args.precision,
                 rotations=args.rotations)
    keep = {}

    def submit(k):
        b, wr, wi, nc = reqs[k]
        n = Hd[b].shape[0]
        X = torch.ones((nc, n), dtype=torch.float64, device=dev).t()
        # the server waits for the fill on torch's stream before it reads X
        keep[k] = (X, srv.submit(Hd[b], wr, wi, X, k))

    # warm-up and saturated throughput (closed loop: the rest of the warm
    # requests at once)
    w0 = min(20, warm // 2)
    for k in range(w0):
        submit(k)
    done = {}
    while len(done) < w0:
        for c in srv.poll(wait_ms=20):
            done[c["tag"]] = c
    t0 = srv.clock()
    for k in range(w0, warm):
        submit(k)
    while len(done) < warm:
        for c in srv.poll(wait_ms=20):
            done[c["tag"]] = c
    sat = (warm - w0) / (srv.clock() - t0)
    rate = 0.7 * sat
    # open loop, Poisson arrivals
    gaps = rng.exponential(1.0 / rate, requests)
    arrive = np.cumsum(gaps)
    t0 = srv.clock()
    nxt, recs = 0, {}
    keep.clear()
    while len(recs) < requests:
        now = srv.clock() - t0
        while nxt < requests and arrive[nxt] <= now:
            submit(warm + nxt)
            nxt += 1
        wait = 5 if nxt >= requests else max(0, min(5, int((arrive[nxt] - now) * 1e3)))
        for c in srv.poll(wait_ms=wait):
            recs[c["tag"]] = c
            keep.pop(c["tag"], None)
    t_end = max(c["t_done"] for c in recs.values())
    t_first = min(c["t_submit"] for c in recs.values())
    lat = [1e3 * (c["t_done"] - c["t_submit"]) for c in recs.values()]
    cols = sum(reqs[k][3] for k in recs)
    status_bad = sum(1 for c in recs.values() if c["status"] != 0)
    fb = sum(c["fallback"] for c in recs.values())
    srv.close()
    out = {
        "workload": "requests on 64 random unreduced Hessenberg matrices, n log-uniform in [128, 8192], "
                    "U{1..n/8} host-eigenvalue shifts (30% complex pairs), all-ones starts; HBM budget 200 GB",
        "requests": requests, "warmup": warm, "precision": args.precision, "nb": args.nb or 128,
        "rotations": args.rotations,
        "p50_ms": round(order_stat(lat, 0.5), 3), "p99_ms": round(order_stat(lat, 0.99), 3),
        "max_ms": round(max(lat), 3),
        "arrival_rate_per_s": round(rate, 2), "saturated_requests_per_s": round(sat, 2),
        "eigenvectors_per_s": round(cols / (t_end - t_first), 2),
        "failed_requests": status_bad,
    }
    if args.precision == 1:
        out["fallback_shifts"] = fb
    return out


def bench_c5(args):
    """The serving workload alone (see serving_run), as its own JSON line."""
    sv = serving_run(args, args.requests, 200)
    line = {
        "metric": "serving p50/p99 request latency (Poisson arrivals at 0.7x saturated throughput)",
        "value": sv["p99_ms"], "unit": "ms (p99)", "n_gpus": 1,
        "steps": args.requests, "warmup": 200, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == 0 else "f64+f32", "data": "synthetic",
        "config": {"workload": sv["workload"], "requests": args.requests, "precision": args.precision,
                   "nb": sv["nb"], "rotations": args.rotations},
    }
    line.update({k: v for k, v in sv.items() if k not in ("workload", "requests", "warmup", "precision", "nb",
                                                         "rotations")})
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--nb", type=int, default=0)
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--rotations", type=int, default=1, choices=[0, 1],
                    help="0: off-diagonal rotations one at a time (bit-identical to the paper's order); "
                         "1: folded into one matrix per tile column and applied on the matrix cores")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["c3", "c4", "c5", "hessenberg"], default="c3",
                    help="c3: the headline single-matrix solve; c4: 512 matrices of uneven order in one "
                         "graph launch (batching); c5: the serving loop under Poisson arrivals")
    ap.add_argument("--requests", type=int, default=2000, help="c5: open-loop arrivals")
    ap.add_argument("--share-min-far", type=int, default=0,
                    help="c3: far-tile blocks from which a step uses the CU-sharing critical kernel (0 = default)")
    ap.add_argument("--cols-per-block", type=int, default=0, help="c3: far-block width (0 = default)")
    ap.add_argument("--hess-n", type=int, default=8000, help="hessenberg: matrix order")
    ap.add_argument("--hess-cols", type=int, default=1000, help="hessenberg: vectors back-transformed")
    ap.add_argument("--serving-requests", type=int, default=300,
                    help="c3: Poisson arrivals of the serving sub-measurement (0 = skip it)")
    ap.add_argument("--one-form", action="store_true",
                    help="c3: time only the form given by --rotations")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run only a plain device copy of known size (counter calibration)")
    ap.add_argument("--ingest-pmc", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="write profiles/traffic_c3.json from rocprofv3 counter_collection.csv files")
    ap.add_argument("--ingest-mfma", nargs=2, metavar=("PMC_CSV", "KERNEL_STATS_CSV"),
                    help="write profiles/mfma_c3.json from a counter run and the kernel statistics of a trace run")
    args = ap.parse_args()
    if args.ingest_mfma:
        ingest_mfma(*args.ingest_mfma)
        return
    if args.ingest_pmc:
        ingest_pmc(*args.ingest_pmc, COPY_BYTES)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the path shards over shifts with no communication, "
              "and this build runs and reports a single MI355X only (use --gpus 1).", flush=True)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    if args.workload == "c4":
        bench_c4(args)
        return
    if args.workload == "c5":
        bench_c5(args)
        return
    if args.workload == "hessenberg":
        bench_hessenberg(args)
        return

    import numpy as np
    import torch

    from paper_2101_05063_amd import Solver
    from workloads import generators as g

    c = g.config_c3()
    H, wr, wi, B = c["H"], c["wr"], c["wi"], c["B"]
    n, m = H.shape[0], len(wr)
    dev = torch.device("cuda:0")
    Hd = torch.from_numpy(np.ascontiguousarray(H.T)).to(dev).t()
    Bd = torch.from_numpy(np.ascontiguousarray(B.T)).to(dev).t()
    solver = Solver(0)
    nb = args.nb
    # the tile size the library chooses (same rule as the host planner)
    nbv = nb if nb in (64, 128) else (128 if n >= 2048 else 64)
    fl = table1_flops(n, nbv, wi)
    forms = [args.rotations] + ([1 - args.rotations] if args.precision == 0 and not args.one_form else [])
    res = {rot: run_c3_form(solver, Hd, Bd, wr, wi, nb, nbv, rot, fl, args) for rot in forms}
    head = res[args.rotations]
    ms, kern = head["ms"], head["kernels"]
    dom = max(kern, key=lambda k: kern[k]["ms_per_step"])
    dk = kern[dom]
    roof = {"kernel": dk["kernel"], "bound": "alu", "achieved": dk["achieved_tflops"],
            "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": dk["frac_fp64_peak"],
            "traffic": load_traffic(dk["kernel"]),
            "avg_launch_ms": dk["avg_launch_ms"], "launches_per_step": dk["launches_per_step"],
            "flops_per_launch": dk["flops_per_launch"]}
    line = {
        "metric": "eigenvectors/s (n=8000, m=1000; + % FP64 MFMA peak of the level-3 update)",
        "value": round(m / (ms * 1e-3), 2), "unit": "eigenvectors/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == 0 else "f64+f32", "data": "synthetic",
        "config": {"workload": "graded random unreduced Hessenberg n=8000, 1000 real eigenvalue shifts, "
                               "all-ones starts (D_ii = 10^(300 i/n))",
                   "n": n, "m": m, "nb": nbv, "precision": args.precision, "rotations": args.rotations,
                   "graph": head["graph"]},
        "ms_per_step_kernel_by_kernel": head["ms_eager"],
        "ms_per_step_with_kernel_events": head["ms_prof"],
        "roofline": roof,
        "kernels": kern,
        "level3_update": head["update"],
        "path_tflops": round(fl["total"] / (ms * 1e-3) / 1e12, 3),
        "phases_ms_per_step": head["phases"],
        "converged_fraction": head["converged_fraction"],
        "scale_exp_range": head["scale_exp_range"],
    }
    if args.precision == 1:
        line["fallback_shifts"] = solver.fallback_count()
    for rot in forms[1:]:
        o = res[rot]
        line["one_at_a_time_form" if rot == 0 else "level3_form"] = {
            "rotations": rot, "value": round(m / (o["ms"] * 1e-3), 2), "unit": "eigenvectors/s",
            "ms_per_step": o["ms"], "ms_per_step_kernel_by_kernel": o["ms_eager"], "kernels": o["kernels"],
            "level3_update": o["update"], "converged_fraction": o["converged_fraction"]}
    solver.close()
    if not args.no_cpu_baseline:
        cores = len(os.sched_getaffinity(0))
        base, sel, ref = cpu_reference_c3(c, args.cpu_seconds, cores)
        line["cpu_baseline"] = base
        # every form's results against the reference on the same sample
        err = {}
        for rot in forms:
            o = res[rot]
            err[f"rotations={rot}"] = error_vs_reference_c3(o["Y"], o["E"], o["mu"], o["info"], sel, ref, wi)
        line["error_vs_reference"] = err
    if args.serving_requests > 0 and args.precision == 0:
        line["serving"] = serving_run(args, args.serving_requests, 100)
    print(json.dumps(line), flush=True)


def mfma_counters():
    """MFMA-busy fractions per kernel from the committed counter run (valid
    only for the kernel sources it was taken on), or {}."""
    if not os.path.exists(MFMA_FILE):
        return {}
    d = json.load(open(MFMA_FILE))
    if d.get("kernel_source_hash") != kernel_source_hash():
        return {}
    return d.get("kernels", {})


def run_c3_form(solver, Hd, Bd, wr, wi, nb, nbv, rotations, fl, args):
    """K solves of C3 in one form of ReduceOffdiag, timed three ways: replayed
    from the library's captured graph (the figure reported), kernel by
    kernel, and kernel by kernel with HIP timing events attached to every
    step-kernel dispatch (the kernel durations)."""
    import numpy as np
    import torch
    m, n = len(wr), Hd.shape[0]
    # preallocate every in/out buffer: the timed regions hold solves only
    Xw = [Bd.clone() for _ in range(max(args.warmup, 1))]
    Xs = [Bd.clone() for _ in range(args.steps)]
    # the FP32 variant is launched kernel by kernel: it has a host decision inside
    graph = 1 if args.precision == 0 else -1

    def timed(graph, prof):
        # the solve overwrites X with the result: fresh right-hand sides for
        # every pass, outside the timed region
        for A in Xw + Xs:
            A.copy_(Bd)
        torch.cuda.synchronize()
        for k in range(args.warmup):
            solver.dhsrq3(Hd, wr, wi, Xw[k], nb=nb, precision=args.precision, graph=graph, rotations=rotations,
                          share_min_far=args.share_min_far, cols_per_block=args.cols_per_block)
        torch.cuda.synchronize()
        if prof:
            solver.profile(True)
            solver.profile_read()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = []
        for k in range(args.steps):
            outs.append(solver.dhsrq3(Hd, wr, wi, Xs[k], nb=nb, precision=args.precision, graph=graph,
                                      rotations=rotations, share_min_far=args.share_min_far,
                                      cols_per_block=args.cols_per_block))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pr = None
        if prof:
            pr = solver.profile_read()
            solver.profile(False)
        return (t1 - t0) * 1e3 / args.steps, outs, pr

    ms, outs, _ = timed(graph, False)
    E, mu, info = (t.cpu().numpy() for t in outs[-1][:3])
    Y = Xs[-1].t().contiguous().cpu().numpy().T
    ms_eager, _, _ = timed(-1, False)
    ms_prof, _, prof = timed(-1, True)
    l3 = args.precision == 0 and rotations == 1
    f32 = "true" if args.precision == 1 else "false"
    kern = {}
    for kind in ("crit", "far"):
        ms_k, launches = prof[kind]
        per_solve = ms_k / args.steps
        if kind == "far":
            # the far-block width: the library default (32 columns in the level-3 form, 64 otherwise)
            cbv = args.cols_per_block if args.cols_per_block in (32, 64) else (32 if l3 else 64)
            name = f"hsrq::k_far3<{nbv}, {cbv}>" if l3 else f"hsrq::k_far<{nbv}, {f32}>"
        else:
            # steps with many far-tile blocks use the variant that shares its CU
            tmpl = f"<{nbv}, {f32}, {'true' if l3 else 'false'}>"
            name = f"hsrq::k_crit{tmpl} + hsrq::k_crit_sh{tmpl}"
        ach = fl[kind] / (per_solve * 1e-3) / 1e12 if per_solve > 0 else 0.0
        kern[kind] = {"kernel": name, "ms_per_step": round(per_solve, 4),
                      "launches_per_step": launches / args.steps,
                      "avg_launch_ms": round(ms_k / launches, 5) if launches else None,
                      "flops_per_launch": fl[kind] / (launches / args.steps) if launches else None,
                      "achieved_tflops": round(ach, 3), "frac_fp64_peak": round(ach / PEAK_FP64_TFLOPS, 4)}
    # the level-3 update in the far-tile kernel: its matrix-core flops (the
    # update product, and in the level-3 form also the rotation product with
    # the same H tile) over that kernel's own time
    far_ms = prof["far"][0] / args.steps
    mfma = fl["far_update"] * (2.0 if l3 else 1.0)
    upd = {"kernel": kern["far"]["kernel"], "update_flops_per_step": fl["update"],
           "far_kernel_mfma_flops_per_step": mfma,
           "far_kernel_mfma_tflops": round(mfma / (far_ms * 1e-3) / 1e12, 3) if far_ms > 0 else None,
           "frac_fp64_mfma_peak": round(mfma / (far_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4) if far_ms > 0 else None}
    cnt = mfma_counters().get(kern["far"]["kernel"])
    if cnt:
        upd["mfma_busy_from_counters"] = cnt.get("mfma_busy")
    return {"ms": round(ms, 4), "ms_eager": round(ms_eager, 4), "ms_prof": round(ms_prof, 4), "graph": graph == 1,
            "kernels": kern, "update": upd,
            "phases": {k: round(v[0] / args.steps, 4) for k, v in prof.items()},
            "converged_fraction": float((info == 0).mean()),
            "scale_exp_range": [int(E.min()), int(E.max())], "Y": Y, "E": E, "mu": mu, "info": info}


if __name__ == "__main__":
    main()
