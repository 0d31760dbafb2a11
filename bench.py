#!/usr/bin/env python3
"""Throughput of the batched 3x3 symmetric eigendecomposition on one MI355X.

Default workload (one step = one pass of the 3x3 forward path over the batch):
2^24 float32 3x3 matrices Q diag(lam) Q^T (Haar Q, lam ~ U[-1,1]^3, 10 %
near-degenerate with relative gaps log-uniform in [1e-7, 1e-3], 1 % exactly
repeated, diagonal and zero matrices), structure-of-arrays planes resident in
HBM; outputs lam, D and the angles.  The float32 path computes the cubic step
in float64, the angle solve in float32, checks every D in float64 and refines
the failing matrices in float64 inside the same kernel.

Printed: one JSON line with matrices/s, the roofline of the kernel (HBM,
algorithmic bytes 84 per matrix), the CPU oracle's throughput on the host cores,
the float64 GPU path on the same matrices, accuracy on a sample, the median
and minimum of single launches, and the throughput at two further seeds of the
same recipe (timed step only; --seeds).

Other workloads for measurement (--workload): mixed (2^26 mixed 2x2/3x3 in
1024 groups, one persistent launch replayed from a HIP graph), grad (2^22
forward + backward), field (256^3 array-of-structures tensor field, forward +
backward), copy (a device copy of known size, for counter calibration).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_PEAK_TLANE = 256 * 64 * 2.4e9 / 1e12   # 39.3 T lane-instructions/s
BYTES_3X3_F32 = 84      # 24 in + 60 out (lam 12, D 36, phi 12)
BYTES_3X3_F64 = 168
BYTES_3X3_LAM_F32 = 36  # eigenvalues-only mode: 24 in + 12 out (lam)
BYTES_2X2_F32 = 40      # 12 in + 28 out (lam 8, D 16, phi 4)
BYTES_BWD_F32 = 120     # lam 12 + D 36 + glam 12 + gD 36 in, gA 24 out


def _source_digest():
    """sha256 of the HIP sources (csrc/*.hip, *.hpp), to tie stored counter
    readings to the kernels they were taken on."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1306_6291_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if not f.endswith((".hip", ".hpp")):
            continue
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def _stored_profile(name):
    """Key/value lines of profiles/<name>.txt (written from rocprofv3 runs), or
    None when the file is missing or the kernel sources have changed since
    the counters were taken (its source_digest no longer matches)."""
    path = os.path.join(ROOT, "profiles", f"{name}.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    if rec.get("source_digest") != _source_digest():
        return None
    return rec


def _stored_traffic(name):
    """HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE runs, or None."""
    rec = _stored_profile(f"{name}_traffic")
    try:
        return float(rec["hbm_bytes_per_launch"]) if rec else None
    except (KeyError, ValueError):
        return None


def _stored_valu(name):
    """VALU instructions per dispatch (SQ_INSTS_VALU, wave instructions) from
    the counter run, or None."""
    rec = _stored_profile(f"{name}_valu")
    try:
        return float(rec["SQ_INSTS_VALU_per_dispatch"]) if rec else None
    except (KeyError, ValueError):
        return None


def _cpu_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _time_steps(fn, steps, warmup, torch):
    """Warm up, then time exactly `steps` calls between HIP events recorded on
    the current stream (the stream the library launches on)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    for _ in range(steps):
        fn()
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def _step_stats(fn, steps, torch):
    """Per-step durations (ms) of `steps` further calls, each between its own
    pair of HIP events on the current stream: median and minimum.  Run after
    the timed region, so the headline mean is not affected."""
    st = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record(st)
        fn()
        b.record(st)
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in ev])
    return {"median": float(np.median(t)), "min": float(t.min()), "steps": steps}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _accuracy(P32, out, n_sample, torch, seed=0):
    """Accuracy of a result, without the oracle: residual max_k ||A d_k -
    lam_k d_k|| / ||A||_F and max |D^T D - I| over every matrix (float64 on the
    GPU, plane by plane, in chunks), and |delta lam| / ||A||_F against LAPACK
    (numpy eigvalsh) on a random sample."""
    n = P32.shape[1]
    res_max = 0.0
    orth_max = 0.0
    chunk = 1 << 22
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        a11, a22, a33, a12, a13, a23 = torch.from_numpy(P32[:, s:e]).to("cuda", torch.float64)
        A = ((a11, a12, a13), (a12, a22, a23), (a13, a23, a33))
        D = out["D"][:, s:e].to(torch.float64)
        L = out["lam"][:, s:e].to(torch.float64)
        fro = torch.sqrt(a11 * a11 + a22 * a22 + a33 * a33 + 2 * (a12 * a12 + a13 * a13 + a23 * a23))
        fro = torch.where(fro > 0, fro, torch.ones_like(fro))
        for k in range(3):
            col = (D[k], D[3 + k], D[6 + k])
            r2 = sum((A[i][0] * col[0] + A[i][1] * col[1] + A[i][2] * col[2] - L[k] * col[i]) ** 2
                     for i in range(3))
            res_max = max(res_max, float((torch.sqrt(r2) / fro).max()))
            for j in range(k, 3):
                dot = D[j] * D[k] + D[3 + j] * D[3 + k] + D[6 + j] * D[6 + k]
                orth_max = max(orth_max, float((dot - (1.0 if j == k else 0.0)).abs().max()))
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(n, size=min(n_sample, n), replace=False))
    P64 = P32[:, idx].astype(np.float64)
    a11, a22, a33, a12, a13, a23 = P64
    A = np.stack([np.stack([a11, a12, a13], 1), np.stack([a12, a22, a23], 1),
                  np.stack([a13, a23, a33], 1)], 1)
    ref = np.linalg.eigvalsh(A)
    lam = np.sort(out["lam"][:, idx].cpu().numpy().astype(np.float64).T, axis=1)
    fro = np.sqrt((A * A).sum((1, 2)))
    err = np.abs(lam - ref).max(1) / np.where(fro > 0, fro, 1)
    return {"residual_max": res_max, "orth_max": orth_max, "lam_err_max_vs_lapack": float(err.max()),
            "lam_sample": int(idx.size)}


def bench_precision(args, torch, ksym, synth):
    n = args.n or (1 << 24)
    t0 = time.perf_counter()
    P32 = synth.make_precision(n)
    print(f"[bench] generated {n} matrices in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    A = torch.from_numpy(P32).to(dev)
    out = {"lam": torch.empty((3, n), device=dev), "D": torch.empty((9, n), device=dev),
           "phi": torch.empty((3, n), device=dev)}
    opts = ksym.tuned_opts("eig3", ksym.F32)

    def step():
        ksym.eig3(A, opts=opts, out=out)

    ms, wall = _time_steps(step, args.steps, args.warmup, torch)
    value = n / (ms * 1e-3)
    achieved = BYTES_3X3_F32 * n / (ms * 1e-3) / 1e9
    per_step = _step_stats(step, min(args.steps, 50), torch)
    # refined fraction and flags, one extra untimed call with the counters
    ws = ksym.workspace()
    flags = torch.empty((n,), dtype=torch.uint8, device=dev)
    ksym.eig3(A, opts=opts, out=dict(out, flags=flags), ws=ws)
    torch.cuda.synchronize()
    refined = int(ws[0].item())
    res = {"ms": ms, "wall": wall, "value": value, "achieved": achieved, "refined": refined, "n": n,
           "opts": opts.as_dict(), "per_step": per_step,
           "input_sha256": hashlib.sha256(np.ascontiguousarray(P32).data).hexdigest()[:16]}
    if args.accuracy:
        res["accuracy"] = _accuracy(P32, out, args.accuracy, torch)
    # reduced-output mode on the same matrices: eigenvalues only (no D, no
    # angles), which runs the eigenvalues-only kernel; reported beside the
    # metric, not in it
    lam_only = {"lam": out["lam"]}
    opts_l = ksym.tuned_opts("eig3_lam", ksym.F32)
    ms_l, _ = _time_steps(lambda: ksym.eig3(A, opts=opts_l, out=lam_only), max(3, args.steps // 2),
                          max(2, args.warmup // 2), torch)
    res["lam_only"] = {"value": n / (ms_l * 1e-3), "ms_per_step": ms_l, "bytes_per_matrix": BYTES_3X3_LAM_F32,
                       "achieved_GBs": BYTES_3X3_LAM_F32 * n / (ms_l * 1e-3) / 1e9,
                       "kernel": "k_eig3_lam (outputs lam only)", "block": opts_l.block,
                       "mats_per_lane": opts_l.mats_per_lane, "grid_mult": opts_l.grid_mult}
    # the same recipe at further seeds (timed step only), beside the headline
    if args.seeds > 1 and not args.n:
        vals = [value]
        for k in range(1, args.seeds):
            Pk = synth.make_precision(n, seed=synth.BASE_SEED + 1 + 1000 * k)
            A.copy_(torch.from_numpy(Pk))
            del Pk
            ms_k, _ = _time_steps(step, args.steps, max(20, args.warmup // 4), torch)
            vals.append(n / (ms_k * 1e-3))
        A.copy_(torch.from_numpy(P32))
        res["seeds"] = {"values": vals, "min": min(vals), "max": max(vals),
                        "seeds": [synth.BASE_SEED + 1 + 1000 * k for k in range(args.seeds)]}
    # float64 GPU path on the same matrices
    if not args.no_fp64:
        del out
        A64 = A.double()
        out64 = {"lam": torch.empty((3, n), dtype=torch.float64, device=dev),
                 "D": torch.empty((9, n), dtype=torch.float64, device=dev),
                 "phi": torch.empty((3, n), dtype=torch.float64, device=dev)}
        f64 = {}
        for name, path in (("fp64_fixup", ksym.PATH_FP64_FIXUP), ("fp64_plain", ksym.PATH_FP64_PLAIN)):
            o64 = ksym.tuned_opts("eig3", ksym.F64)
            o64.path = path
            ms64, _ = _time_steps(lambda: ksym.eig3(A64, opts=o64, out=out64), max(3, args.steps // 4),
                                  max(2, args.warmup // 4), torch)
            rec = {"value": n / (ms64 * 1e-3), "ms_per_step": ms64,
                   "achieved_GBs": BYTES_3X3_F64 * n / (ms64 * 1e-3) / 1e9}
            if args.accuracy:
                rec["accuracy"] = _accuracy(P32, out64, args.accuracy, torch)
            f64[name] = rec
        res["fp64"] = f64
        del A64, out64
    if not args.no_cpu:
        import oracle  # CPU baseline leg: the oracle as it stands
        th = _cpu_threads()
        m = min(n, args.cpu_sample)
        P64 = P32[:, :m].astype(np.float64)
        oracle.eig3(P64[:, :1024], threads=1)   # load + warm
        t0 = time.perf_counter()
        oracle.eig3(P64, threads=th)
        dt = time.perf_counter() - t0
        res["cpu"] = {"value": m / dt, "unit": "matrices/s", "cores": th, "kind": "oracle",
                      "sample": f"first {m} matrices of this workload promoted to float64; "
                                f"C float64 oracle of paper §4-§5, {th} host threads, {dt:.2f}s wall",
                      "cpu_model": _cpu_model(), "compiler_flags": " ".join(oracle.CFLAGS)}
    return res


def bench_copy(args, torch):
    """Plain device copy of a known size (counter calibration)."""
    n = 1 << 28   # 1 GiB of float32
    x = torch.ones(n, device="cuda")
    y = torch.empty_like(x)
    ms, _ = _time_steps(lambda: y.copy_(x), args.steps, args.warmup, torch)
    return {"ms": ms, "bytes_read": 4 * n, "bytes_written": 4 * n, "GBs": 8 * n / (ms * 1e-3) / 1e9}


def bench_mixed(args, torch, ksym, synth):
    total = args.n or (1 << 26)
    dev = torch.device("cuda:0")
    sizes, kinds = synth.mixed_group_sizes(total)
    rng = np.random.default_rng(synth.BASE_SEED + 1002)
    groups = []
    bytes_alg = 0
    for s, k in zip(sizes, kinds):
        s = int(s)
        planes = torch.from_numpy(rng.standard_normal((6 if k == 3 else 3, s), dtype=np.float32)).to(dev)
        if k == 3:
            out = {"lam": torch.empty((3, s), device=dev), "D": torch.empty((9, s), device=dev),
                   "phi": torch.empty((3, s), device=dev)}
            bytes_alg += BYTES_3X3_F32 * s
        else:
            out = {"lam": torch.empty((2, s), device=dev), "D": torch.empty((4, s), device=dev),
                   "phi": torch.empty((s,), device=dev)}
            bytes_alg += BYTES_2X2_F32 * s
        groups.append((int(k), planes, out))
    plan = ksym.Plan(groups, opts=ksym.tuned_opts("mixed", ksym.F32))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.capture(stream)
    torch.cuda.synchronize()
    cur = torch.cuda.current_stream()

    def step():
        plan.replay(cur)

    ms, wall = _time_steps(step, args.steps, args.warmup, torch)
    per_step = _step_stats(step, min(args.steps, 50), torch)
    frac2 = float(sizes[kinds == 2].sum()) / total
    return {"ms": ms, "wall": wall, "value": total / (ms * 1e-3), "n": total, "ms_per_step_dist": per_step,
            "achieved": bytes_alg / (ms * 1e-3) / 1e9, "bytes_alg": bytes_alg, "frac2x2": frac2,
            "plan": plan.info(), "refined": int(plan.ws[0].item())}


def bench_grad(args, torch, ksym, synth):
    n = args.n or (1 << 22)
    d = synth.make_grad(n)
    dev = torch.device("cuda:0")
    A = torch.from_numpy(d["planes3"]).to(dev)
    w = torch.from_numpy(d["w"]).to(dev)
    G = torch.from_numpy(d["G"]).to(dev)
    opts = ksym.tuned_opts("eig3_grad", ksym.F32)
    out = {"lam": torch.empty((3, n), device=dev), "D": torch.empty((9, n), device=dev),
           "gap": torch.empty((3, n), device=dev)}
    gA = torch.empty((6, n), device=dev)
    ms_f, _ = _time_steps(lambda: ksym.eig3(A, opts=opts, out=out), args.steps, args.warmup, torch)
    ms_b, _ = _time_steps(lambda: ksym.eig3_backward(out["lam"], out["D"], w, G, gap=out["gap"], out=gA),
                          args.steps, args.warmup, torch)

    def step():   # forward and backward together, one step
        ksym.eig3(A, opts=opts, out=out)
        ksym.eig3_backward(out["lam"], out["D"], w, G, gap=out["gap"], out=gA)

    ms_s, _ = _time_steps(step, args.steps, args.warmup, torch)
    return {"ms_fwd": ms_f, "ms_bwd": ms_b, "ms_step": ms_s, "n": n, "value": n / (ms_s * 1e-3),
            "fwd_GBs": 96 * n / (ms_f * 1e-3) / 1e9, "bwd_GBs": (BYTES_BWD_F32 + 12) * n / (ms_b * 1e-3) / 1e9}


def bench_field(args, torch, ksym, synth):
    nx = args.field_n
    d = synth.make_field(nx, nx, nx)
    n = nx ** 3
    dev = torch.device("cuda:0")
    rec = torch.from_numpy(d["aos"]).to(dev)
    w = torch.from_numpy(d["w"]).to(dev)
    G = torch.from_numpy(d["G"]).to(dev)
    opts = ksym.tuned_opts("eig3_aos", ksym.F32)
    out = {"lam": torch.empty((3, n), device=dev), "D": torch.empty((9, n), device=dev),
           "gap": torch.empty((3, n), device=dev)}
    gA = torch.empty((6, n), device=dev)
    ms_f, _ = _time_steps(lambda: ksym.eig3_aos(rec, opts=opts, out=out), args.steps, args.warmup, torch)
    ms_b, _ = _time_steps(lambda: ksym.eig3_backward(out["lam"], out["D"], w, G, gap=out["gap"], out=gA),
                          args.steps, args.warmup, torch)

    def step():   # forward and backward together, one step
        ksym.eig3_aos(rec, opts=opts, out=out)
        ksym.eig3_backward(out["lam"], out["D"], w, G, gap=out["gap"], out=gA)

    ms_s, _ = _time_steps(step, args.steps, args.warmup, torch)
    return {"ms_fwd": ms_f, "ms_bwd": ms_b, "ms_step": ms_s, "n": n, "value": n / (ms_s * 1e-3),
            "fwd_GBs": 96 * n / (ms_f * 1e-3) / 1e9, "bwd_GBs": (BYTES_BWD_F32 + 12) * n / (ms_b * 1e-3) / 1e9}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200,
                    help="untimed launches first (the GPU reaches its steady clock after ~0.1 s of work)")
    ap.add_argument("--workload", default="precision",
                    choices=["precision", "mixed", "grad", "field", "copy"])
    ap.add_argument("--n", type=int, default=0, help="override the batch size")
    ap.add_argument("--field-n", type=int, default=256)
    ap.add_argument("--cpu-sample", type=int, default=1 << 24)
    ap.add_argument("--accuracy", type=int, default=1 << 16,
                    help="matrices sampled for the eigenvalue check of the accuracy report (0 = skip)")
    ap.add_argument("--seeds", type=int, default=3,
                    help="precision workload: also time the recipe at this many seeds in all "
                         "(the first is the headline's), to show the spread")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the matrices are independent, and the library "
              "has no multi-GPU path. Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    import paper_1306_6291_amd as ksym
    import synth

    base = {"metric": "3x3 sym eigendecomps/sec, FP32+fixup vs FP64 at stated err; % HBM/VALU peak",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "data": "synthetic"}

    if args.workload == "copy":
        r = bench_copy(args, torch)
        print(json.dumps({"workload": "copy", **r}))
        return

    if args.workload == "precision":
        r = bench_precision(args, torch, ksym, synth)
        traffic = _stored_traffic("eig3_f32_precision")
        valu = _stored_valu("eig3_f32_precision")
        line = dict(base)
        line.update({
            "value": r["value"], "unit": "matrices/s", "ms_per_step": r["ms"], "dtype": "f32",
            "config": {"workload": "precision: 2^24 float32 3x3 Q diag(lam) Q^T, Haar Q, lam~U[-1,1]^3, "
                                   "10% rel. gaps logU[1e-7,1e-3], 1% repeated, diagonal + zero matrices; "
                                   "SoA planes in HBM; outputs lam, D, angles",
                       "n": r["n"], "path": "float32 angle solve, float64 cubic step, float64 check + refinement",
                       "block": r["opts"]["block"], "mats_per_lane": r["opts"]["mats_per_lane"],
                       "grid_mult": r["opts"]["grid_mult"], "tau_res": r["opts"]["tau_res"],
                       "refined_fraction": r["refined"] / r["n"], "input_sha256": r["input_sha256"]},
            "ms_per_step_dist": r["per_step"],
            "roofline": {"bound": "hbm", "achieved": r["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": r["achieved"] / HBM_PEAK_GBS,
                         "traffic": traffic, "traffic_unit": "HBM bytes per launch (rocprofv3 counters)",
                         "algorithmic_bytes": BYTES_3X3_F32 * r["n"],
                         "kernel": "k_eig3<float, FP32_FIXUP>", "bytes_per_matrix": BYTES_3X3_F32},
        })
        if valu is not None:
            # VALU side of the same kernel: wave instructions per launch (rocprofv3
            # SQ_INSTS_VALU) x 64 lanes / launch time, against 256 CUs x 64 lanes x 2.4 GHz
            rate = valu * 64 / (r["ms"] * 1e-3) / 1e12
            line["valu"] = {"achieved": rate, "peak": VALU_PEAK_TLANE, "unit": "T lane-instr/s",
                            "frac": rate / VALU_PEAK_TLANE, "instr_per_matrix": valu * 64 / r["n"]}
        if "cpu" in r:
            line["cpu_baseline"] = r["cpu"]
        if "fp64" in r:
            line["fp64_path"] = r["fp64"]
        if "lam_only" in r:
            line["eigenvalues_only"] = r["lam_only"]
        if "seeds" in r:
            line["seed_spread"] = r["seeds"]
        if "accuracy" in r:
            line["accuracy"] = r["accuracy"]
        print(json.dumps(line), flush=True)
        return

    fn = {"mixed": bench_mixed, "grad": bench_grad, "field": bench_field}[args.workload]
    r = fn(args, torch, ksym, synth)
    print(json.dumps({"workload": args.workload, **r}), flush=True)


if __name__ == "__main__":
    main()
