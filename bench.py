#!/usr/bin/env python3
"""Throughput of the batched 3x3 symmetric eigendecomposition on one MI355X.

Default workload (one step = one pass of the 3x3 forward path over the batch):
2^24 float32 3x3 matrices Q diag(lam) Q^T (Haar Q, lam ~ U[-1,1]^3, 10 %
near-degenerate with relative gaps log-uniform in [1e-7, 1e-3], 1 % exactly
repeated, diagonal and zero matrices), structure-of-arrays planes resident in
HBM; outputs lam, D and the angles.  The float32 path computes the cubic step
in float64, the angle solve in float32, checks every D and refines the
failing matrices in float64 inside the same kernel.

Order: the inputs are generated and copied to the device; one forward with
the flags and counters runs and its result is checked (eigenvalues against
LAPACK on a sample, residual and orthogonality of every matrix on the GPU);
the steady-state leg (at least 0.2 s of untimed launches, then the timed
steps) follows, then the warmup steps and the timed steps of the headline,
between two counter-reset launches that mark them in a kernel trace.

Printed: one JSON line with matrices/s, the roofline of the kernel (HBM,
algorithmic bytes 84 per matrix), the CPU oracle's throughput on the host
cores, the float64 GPU paths on the same matrices, the accuracy, the median
and minimum of single launches, a steady-state figure taken after at least
0.2 s of further launches, the reduced-output modes (eigenvalues only;
eigenvalues and angles), the throughput at two further seeds of the same
recipe, and the other workloads of the library (below), each with its
algorithmic bytes and fraction of the HBM roof.

Other workloads (--workload for a line of their own; in the default line
under "workloads"): mixed (2^26 mixed 2x2/3x3 in 1024 groups, one persistent
launch replayed from a HIP graph), grad (2^22 forward + backward), field
(256^3 array-of-structures tensor field, forward + backward), eig2 (2^24
float32 2x2), copy (a device copy of known size, for counter calibration).
"""

from __future__ import annotations

import argparse
import hashlib
import re
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
BYTES_3X3_LAMPHI_F32 = 48   # eigenvalues and angles, no D: 24 in + 24 out
BYTES_2X2_F32 = 40      # 12 in + 28 out (lam 8, D 16, phi 4)
BYTES_BWD_F32 = 120     # lam 12 + D 36 + glam 12 + gD 36 in, gA 24 out


def _source_digest():
    """sha256 of the HIP sources (csrc/*.hip, *.hpp) with comments and
    whitespace removed, to tie stored counter readings to the code they were
    taken on (an edit of a comment leaves the readings valid)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1306_6291_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if not f.endswith((".hip", ".hpp")):
            continue
        with open(os.path.join(d, f), encoding="utf-8") as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(f.encode())
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def _stored_profile(name):
    """Key/value lines of profiles/<name>.txt (summaries of rocprofv3 runs),
    or None when the file is missing or the kernel sources have changed since
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


def _stored_float(name, key):
    rec = _stored_profile(name)
    try:
        return float(rec[key]) if rec else None
    except (KeyError, ValueError):
        return None


def _stored_traffic(name):
    """HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE runs, or None."""
    return _stored_float(name, "hbm_bytes_per_launch")


def _stored_valu(name):
    """VALU instructions per dispatch (SQ_INSTS_VALU, wave instructions) from
    the counter run, or None."""
    return _stored_float(name, "SQ_INSTS_VALU_per_dispatch")


def _counters(name, n):
    """The stored counter figures of one kernel on one workload: HBM bytes
    per launch and VALU lane instructions per matrix (None where absent or
    stale)."""
    t, v = _stored_traffic(name), _stored_valu(name)
    return {"traffic": t, "valu_lane_instr_per_matrix": v * 64 / n if v is not None else None,
            "profile": f"profiles/{name}.txt"}


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


def _warm(fn, torch, seconds):
    """Untimed calls for at least `seconds` of wall time (the GPU's clocks
    rise over about 0.1 s of work)."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(8):
            fn()
        torch.cuda.synchronize()


def _timed_after_warm(fn, steps, torch, seconds=0.2):
    """Mean ms of `steps` calls after at least `seconds` of untimed calls."""
    _warm(fn, torch, seconds)
    ms, _ = _time_steps(fn, steps, 0, torch)
    return ms


def _roof(bytes_per_launch, ms):
    gbs = bytes_per_launch / (ms * 1e-3) / 1e9
    return {"achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS}


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
    """Accuracy of a result, without the oracle: |delta lam| / ||A||_F against
    LAPACK (numpy eigvalsh) on a random sample (host), then the residual
    max_k ||A d_k - lam_k d_k|| / ||A||_F and max |D^T D - I| over every
    matrix (float64 on the GPU, plane by plane, in chunks) -- the device
    part last, so that a timed region following it finds the GPU busy."""
    n = P32.shape[1]
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
    res_max = 0.0
    orth_max = 0.0
    chunk = 1 << 22
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        a11, a22, a33, a12, a13, a23 = torch.from_numpy(P32[:, s:e]).to("cuda", torch.float64)
        Am = ((a11, a12, a13), (a12, a22, a23), (a13, a23, a33))
        D = out["D"][:, s:e].to(torch.float64)
        L = out["lam"][:, s:e].to(torch.float64)
        f = torch.sqrt(a11 * a11 + a22 * a22 + a33 * a33 + 2 * (a12 * a12 + a13 * a13 + a23 * a23))
        f = torch.where(f > 0, f, torch.ones_like(f))
        for k in range(3):
            col = (D[k], D[3 + k], D[6 + k])
            r2 = sum((Am[i][0] * col[0] + Am[i][1] * col[1] + Am[i][2] * col[2] - L[k] * col[i]) ** 2
                     for i in range(3))
            res_max = max(res_max, float((torch.sqrt(r2) / f).max()))
            for j in range(k, 3):
                dot = D[j] * D[k] + D[3 + j] * D[3 + k] + D[6 + j] * D[6 + k]
                orth_max = max(orth_max, float((dot - (1.0 if j == k else 0.0)).abs().max()))
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

    # the result is checked first: one call with the flags and counters, then
    # the accuracy of every matrix (on the GPU) and of a sample (LAPACK)
    ws = ksym.workspace()
    flags = torch.empty((n,), dtype=torch.uint8, device=dev)
    ksym.eig3(A, opts=opts, out=dict(out, flags=flags), ws=ws)
    torch.cuda.synchronize()
    refined = int(ws[0].item())
    res = {"refined": refined, "n": n, "opts": opts.as_dict(),
           "input_sha256": hashlib.sha256(np.ascontiguousarray(P32).data).hexdigest()[:16]}
    if args.accuracy:
        res["accuracy"] = _accuracy(P32, out, args.accuracy, torch)
    del flags
    print("[bench] accuracy checked; timing", file=sys.stderr, flush=True)
    # steady state first: K steps after at least 0.2 s of untimed launches
    # (the GPU's clocks need about that long under this load to leave their
    # idle state; a short warmup after idle host work measures the ramp)
    ms_ss = _timed_after_warm(step, args.steps, torch)
    res["steady"] = dict({"ms_per_step": ms_ss, "value": n / (ms_ss * 1e-3), "steps": args.steps,
                          "after": "at least 0.2 s of untimed launches"}, **_roof(BYTES_3X3_F32 * n, ms_ss))
    # the headline: W warmup steps, then exactly K timed steps, between two
    # counter-reset launches that mark the region in a kernel trace
    marker = ksym.workspace()
    ksym.zero_counters(marker)
    ms, wall = _time_steps(step, args.steps, args.warmup, torch)
    ksym.zero_counters(marker)
    res.update({"ms": ms, "wall": wall, "value": n / (ms * 1e-3),
                "achieved": BYTES_3X3_F32 * n / (ms * 1e-3) / 1e9})
    res["per_step"] = _step_stats(step, min(args.steps, 50), torch)
    # reduced-output modes on the same matrices, reported beside the metric:
    # eigenvalues only (no D, no angles: the eigenvalues-only kernel) and
    # eigenvalues and angles (no D: the full kernel, D kept in registers)
    lam_only = {"lam": out["lam"]}
    opts_l = ksym.tuned_opts("eig3_lam", ksym.F32)
    ms_l = _timed_after_warm(lambda: ksym.eig3(A, opts=opts_l, out=lam_only), args.steps, torch)
    res["lam_only"] = dict({"value": n / (ms_l * 1e-3), "ms_per_step": ms_l,
                            "bytes_per_matrix": BYTES_3X3_LAM_F32, "kernel": "k_eig3_lam (outputs lam only)",
                            "block": opts_l.block, "mats_per_lane": opts_l.mats_per_lane,
                            "grid_mult": opts_l.grid_mult, **_counters("eig3_lam_precision", n)},
                           **_roof(BYTES_3X3_LAM_F32 * n, ms_l))
    lam_phi = {"lam": out["lam"], "phi": out["phi"]}
    opts_lp = ksym.tuned_opts("eig3_lamphi", ksym.F32)
    ms_lp = _timed_after_warm(lambda: ksym.eig3(A, opts=opts_lp, out=lam_phi), args.steps, torch)
    res["lam_phi"] = dict({"value": n / (ms_lp * 1e-3), "ms_per_step": ms_lp,
                           "bytes_per_matrix": BYTES_3X3_LAMPHI_F32,
                           "kernel": "k_eig3<float> with no D planes (lam and angles stored)",
                           "block": opts_lp.block, "mats_per_lane": opts_lp.mats_per_lane,
                           "grid_mult": opts_lp.grid_mult, **_counters("eig3_lamphi_precision", n)},
                          **_roof(BYTES_3X3_LAMPHI_F32 * n, ms_lp))
    # the same recipe at further seeds (timed step only), beside the headline
    if args.seeds > 1 and not args.n:
        vals = [n / (ms_ss * 1e-3)]
        for k in range(1, args.seeds):
            Pk = synth.make_precision(n, seed=synth.BASE_SEED + 1 + 1000 * k)
            A.copy_(torch.from_numpy(Pk))
            del Pk
            vals.append(n / (_timed_after_warm(step, args.steps, torch) * 1e-3))
        A.copy_(torch.from_numpy(P32))
        res["seeds"] = {"values": vals, "min": min(vals), "max": max(vals),
                        "seeds": [synth.BASE_SEED + 1 + 1000 * k for k in range(args.seeds)],
                        "timing": "steady state (after at least 0.2 s of untimed launches)"}
    # float64 GPU paths on the same matrices, as many steps as the headline
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

            def step64():
                ksym.eig3(A64, opts=o64, out=out64)

            step64()
            torch.cuda.synchronize()
            rec = {}
            if args.accuracy:
                rec["accuracy"] = _accuracy(P32, out64, args.accuracy, torch)
            ms64, _ = _time_steps(step64, args.steps, args.warmup, torch)
            rec.update({"value": n / (ms64 * 1e-3), "ms_per_step": ms64, "steps": args.steps,
                        "warmup": args.warmup})
            rec.update(_roof(BYTES_3X3_F64 * n, ms64))
            rec.update(_counters({"fp64_fixup": "eig3_f64fixup_precision",
                                  "fp64_plain": "eig3_f64plain_precision"}[name], n))
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


def _timed(fn, args, torch):
    """A secondary workload's timing: at least 0.2 s of untimed calls, the
    warmup steps, then the timed steps (mean ms)."""
    _warm(fn, torch, 0.2)
    ms, _ = _time_steps(fn, args.steps, args.warmup, torch)
    return ms


def bench_mixed(args, torch, ksym, synth):
    total = args.n or (1 << 26)
    dev = torch.device("cuda:0")
    sizes, kinds = synth.mixed_group_sizes(total)
    rng = np.random.default_rng(synth.BASE_SEED + 1002)
    groups = []
    bytes_alg = 0
    for s, k in zip(sizes, kinds):
        s = int(s)
        # each group its own allocation, every plane on a 256-byte boundary
        # (row stride rounded up to 64 elements)
        P = rng.standard_normal((6 if k == 3 else 3, s), dtype=np.float32)
        planes = ksym.line_aligned_planes(P.shape[0], s, device=dev, fill=P)
        if k == 3:
            out = {"lam": ksym.line_aligned_planes(3, s, device=dev), "D": ksym.line_aligned_planes(9, s, device=dev),
                   "phi": ksym.line_aligned_planes(3, s, device=dev)}
            bytes_alg += BYTES_3X3_F32 * s
        else:
            out = {"lam": ksym.line_aligned_planes(2, s, device=dev), "D": ksym.line_aligned_planes(4, s, device=dev),
                   "phi": ksym.line_aligned_planes(1, s, device=dev)[0]}
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

    ms = _timed(step, args, torch)
    per_step = _step_stats(step, min(args.steps, 50), torch)
    frac2 = float(sizes[kinds == 2].sum()) / total
    r = {"workload": "mixed: 2^26 float32 2x2/3x3 (30 % 2x2), N(0,1) entries, 1024 groups of log-uniform sizes, "
                     "every plane 256-byte aligned; one persistent launch replayed from a HIP graph; "
                     "outputs lam, D, angles",
         "kernel": "k_mixed", "value": total / (ms * 1e-3), "unit": "matrices/s", "ms_per_step": ms, "n": total,
         "ms_per_step_dist": per_step, "bytes_per_launch": bytes_alg, "frac2x2": frac2, "plan": plan.info(),
         "refined": int(plan.ws[0].item()), "opts": plan.opts.as_dict(), **_counters("mixed", total)}
    r.update(_roof(bytes_alg, ms))
    plan.close()
    return r


def bench_eig2(args, torch, ksym, synth):
    n = args.n or (1 << 24)
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(synth.BASE_SEED + 1005)
    A = torch.from_numpy(rng.uniform(-1.0, 1.0, size=(3, n)).astype(np.float32)).to(dev)
    out = {"lam": torch.empty((2, n), device=dev), "D": torch.empty((4, n), device=dev),
           "phi": torch.empty((n,), device=dev)}
    opts = ksym.tuned_opts("eig2", ksym.F32)

    def step():
        ksym.eig2(A, opts=opts, out=out)

    ms = _timed(step, args, torch)
    r = {"workload": "eig2: 2^24 float32 2x2, entries U[-1,1]; outputs lam, D, angle", "kernel": "k_eig2",
         "value": n / (ms * 1e-3), "unit": "matrices/s", "ms_per_step": ms, "n": n,
         "bytes_per_matrix": BYTES_2X2_F32, "opts": opts.as_dict(), **_counters("eig2", n)}
    r.update(_roof(BYTES_2X2_F32 * n, ms))
    return r


def _fwd_bwd(args, torch, ksym, fwd, out, w, G, n, label, kernels, opts, prof):
    """Forward, backward and both as one step of a differentiation workload."""
    gA = torch.empty((6, n), device=out["lam"].device)

    def bwd():
        ksym.eig3_backward(out["lam"], out["D"], w, G, gap=out["gap"], out=gA)

    def step():
        fwd()
        bwd()

    ws = ksym.workspace()
    fwd(ws)
    torch.cuda.synchronize()
    refined = int(ws[0].item())
    ms_f = _timed(fwd, args, torch)
    ms_b = _timed(bwd, args, torch)
    ms_s = _timed(step, args, torch)
    fb, bb = BYTES_3X3_F32, BYTES_BWD_F32 + 12   # forward: lam, D and the gaps; backward with the gaps
    r = {"workload": label, "kernels": kernels, "value": n / (ms_s * 1e-3), "unit": "matrices/s (forward + backward)",
         "ms_per_step": ms_s, "n": n, "refined_fraction": refined / n, "opts": opts.as_dict(),
         "bytes_per_matrix": {"forward": fb, "backward": bb, "step": fb + bb},
         "forward": dict({"ms": ms_f, **_counters(f"{prof}_fwd", n)}, **_roof(fb * n, ms_f)),
         "backward": dict({"ms": ms_b, **_counters(f"{prof}_bwd", n)}, **_roof(bb * n, ms_b))}
    r.update(_roof((fb + bb) * n, ms_s))
    return r


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

    def fwd(ws=None):
        ksym.eig3(A, opts=opts, out=out, ws=ws)

    return _fwd_bwd(args, torch, ksym, fwd, out, w, G, n,
                    "grad: 2^22 float32 3x3, N(0,1) entries, relative gap >= 1e-3; loss sum w lam + sum G D; "
                    "forward (lam, D, gaps; float64 pair correction) then the adjoint",
                    "k_eig3<float, GRAD> + k_eig3_bwd", opts, "grad")


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

    def fwd(ws=None):
        ksym.eig3_aos(rec, opts=opts, out=out, ws=ws)

    return _fwd_bwd(args, torch, ksym, fwd, out, w, G, n,
                    f"field: {nx}^3 SPD tensor field, array-of-structures float32 records, eigenvalues "
                    "10^U[-4,-2], smooth rotations, 5 % isotropic; forward (float64 pair correction) then "
                    "the adjoint", "k_eig3<float, AoS, GRAD> + k_eig3_bwd", opts, "field")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200,
                    help="untimed launches first (the GPU reaches its steady clock after ~0.1 s of work)")
    ap.add_argument("--workload", default="precision",
                    choices=["precision", "mixed", "grad", "field", "eig2", "copy"])
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
    # (the 2x2 forward first: after other workloads' allocations it ran 10-17 %
    # slower than in a process of its own)
    ap.add_argument("--workloads", default="eig2,grad,field,mixed",
                    help="precision workload: the other workloads timed into the same line "
                         "(comma-separated from mixed, grad, field, eig2; empty for none)")
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
        if "lam_phi" in r:
            line["eigenvalues_and_angles"] = r["lam_phi"]
        line["steady_state"] = r["steady"]
        if "seeds" in r:
            line["seed_spread"] = r["seeds"]
        if "accuracy" in r:
            line["accuracy"] = r["accuracy"]
        line["timing"] = ("after the accuracy check of one forward and the steady-state leg, "
                          f"{args.warmup} warmup steps, then {args.steps} timed steps between HIP events "
                          "on the launching stream; two k_zero_u32 launches mark the warmup and timed steps "
                          "in a kernel trace")
        # the library's other workloads, each timed on its own inputs
        work = {}
        for name in [w for w in args.workloads.split(",") if w]:
            print(f"[bench] workload {name}", file=sys.stderr, flush=True)
            fn = {"mixed": bench_mixed, "grad": bench_grad, "field": bench_field, "eig2": bench_eig2}[name]
            wargs = argparse.Namespace(**vars(args))
            wargs.n = 0
            work[name] = fn(wargs, torch, ksym, synth)
            torch.cuda.empty_cache()
        if work:
            line["workloads"] = work
        print(json.dumps(line), flush=True)
        return

    fn = {"mixed": bench_mixed, "grad": bench_grad, "field": bench_field, "eig2": bench_eig2}[args.workload]
    r = fn(args, torch, ksym, synth)
    print(json.dumps({"workload": args.workload, **r}), flush=True)


if __name__ == "__main__":
    main()
