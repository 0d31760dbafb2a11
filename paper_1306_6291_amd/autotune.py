"""Autotuner for the ksym kernels: picks block size, matrices per lane, grid
size, the refinement-queue age limit and the refinement threshold tau_res
for each workload on the GPU it runs on, and records them in tuned.json
(read by tuned_opts()).

Stage 1 times every launch shape at the default thresholds (HIP events around
back-to-back launches, median of repeats).  Stage 2 takes the fastest shapes,
tries the refinement thresholds, and keeps the fastest setting whose result
meets the float32 accuracy targets on the whole batch: residual
max_k ||A d_k - lam_k d_k|| <= 1e-5 ||A||_F and |D^T D - I| <= 1e-5 (checked
in float64 on the GPU), and |delta lam| <= 2e-6 ||A||_F against LAPACK on a
random sample.

Workloads (seeded, synthetic; the generators in synth.py):
  eig3/f32       2^24 float32 3x3 of the precision recipe, SoA
  eig3_grad/f32  2^22 float32 3x3, N(0,1) entries, relative gap >= 1e-3,
                 forward with first-order eigenvector certification (tau_vec 1e-4)
  eig3_aos/f32   256^3 SPD tensor field, array-of-structures input, forward
                 with the eigenvector certificate (tau_vec 1e-4): the field is
                 a forward + backward workload
  eig3/f64       the precision recipe promoted to float64, checked path, at
                 the float64 limits (|delta lam| <= 1e-12 ||A||_F against
                 LAPACK, residual <= 2e-11 ||A||_F)
  mixed/f32      2^26 mixed 2x2 / 3x3 in 1024 groups, one graph-captured plan
  eig2/f32       2^24 float32 2x2, U[-1, 1]
  eig3_lam/f32   the precision recipe, eigenvalues only (no D, no angles)

Run on a GPU:  python -m paper_1306_6291_amd.autotune [--kinds eig3/f32,...] [--quick]
"""

from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

import numpy as np
import torch

import paper_1306_6291_amd as ksym

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

RES_TOL = 1e-5
ORTH_TOL = 1e-5
LAM_TOL = 2e-6
# the float64 checked path: eigenvalues to 1e-12 ||A||_F, residual within
# sqrt(3) tau_res of the default tau_res 1e-11
LIMITS_F64 = {"residual_max": 2e-11, "orth_max": 1e-14, "lam_err_max": 1e-12}


def _time(fn, reps=5, steps=20, warmup_ms=200.0):
    """Median over `reps` of the mean time (ms) of `steps` back-to-back calls,
    between HIP events on the current stream.  The calls first run for at
    least warmup_ms of wall time: after host-side work (the accuracy checks)
    the GPU's clocks need about 0.2 s of load to come back up, and a 30 ms
    warm-up read the same launch up to 4 % slow."""
    t0 = time.perf_counter()
    k = 0
    while k < 2 or (time.perf_counter() - t0) * 1e3 < warmup_ms:
        fn()
        k += 1
        if k % 4 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    out = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(steps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1) / steps)
    return float(np.median(out))


def _accuracy3(P, out, sample=1 << 15, seed=0):
    """Residual, orthogonality (every matrix, float64 on the GPU, chunked) and
    eigenvalue error against LAPACK on a sample; relative to ||A||_F."""
    n = P.shape[1]
    res_max = orth_max = 0.0
    chunk = 1 << 22
    eye = torch.eye(3, dtype=torch.float64, device=P.device)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        a11, a22, a33, a12, a13, a23 = P[:, s:e].double()
        A = torch.stack([torch.stack([a11, a12, a13], 1), torch.stack([a12, a22, a23], 1),
                         torch.stack([a13, a23, a33], 1)], 1)
        D = out["D"][:, s:e].double().T.reshape(-1, 3, 3).contiguous()
        L = out["lam"][:, s:e].double().T
        fro = torch.sqrt((A * A).sum((1, 2)))
        r = torch.linalg.vector_norm(torch.bmm(A, D) - D * L[:, None, :], dim=1).amax(1)
        r = torch.where(fro > 0, r / torch.where(fro > 0, fro, torch.ones_like(fro)), r)
        if not bool(torch.isfinite(r).all()):
            return {"residual_max": float("inf"), "orth_max": float("inf"), "lam_err_max": float("inf")}
        res_max = max(res_max, float(r.max()))
        o = (torch.bmm(D.transpose(1, 2).contiguous(), D) - eye).abs()
        orth_max = max(orth_max, float(o.amax()))
    rng = np.random.default_rng(seed)
    idx = torch.from_numpy(np.sort(rng.choice(n, size=min(sample, n), replace=False))).to(P.device)
    Ps = P[:, idx].double().cpu().numpy()
    a11, a22, a33, a12, a13, a23 = Ps
    A = np.stack([np.stack([a11, a12, a13], 1), np.stack([a12, a22, a23], 1), np.stack([a13, a23, a33], 1)], 1)
    ref = np.linalg.eigvalsh(A)
    lam = np.sort(out["lam"][:, idx].double().cpu().numpy().T, axis=1)
    fro = np.sqrt((A * A).sum((1, 2)))
    err = np.abs(lam - ref).max(1) / np.where(fro > 0, fro, 1)
    return {"residual_max": res_max, "orth_max": orth_max, "lam_err_max": float(err.max())}


def _ok(acc, limits=None):
    lim = limits or {"residual_max": RES_TOL, "orth_max": ORTH_TOL, "lam_err_max": LAM_TOL}
    return all(acc[k] <= v for k, v in lim.items())


def _shapes(blocks, mpls, gms, drains):
    return [dict(block=b, mats_per_lane=m, grid_mult=g, drain_tiles=d)
            for b, m, g, d in itertools.product(blocks, mpls, gms, drains)]


def _sweep(run, dtype, shapes, extra, log):
    res = []
    for sh in shapes:
        o = ksym.Opts.defaults(dtype, **sh, **extra)
        try:
            ms = _time(lambda: run(o))
        except ksym.KsymError as e:   # shape not compiled for this kernel
            log(f"  skip {sh}: {e}")
            continue
        res.append((ms, sh))
        log(f"  {ms:.4f} ms  {sh}")
    res.sort(key=lambda r: r[0])
    return res


def _retime_top(res, time_of, log, top=3):
    """Time the `top` fastest shapes of a sweep again (sweep timings differ by
    a few percent between repetitions) and return (ms, shape) of the fastest."""
    log(f"  re-timing the {min(top, len(res))} fastest shapes")
    again = []
    for _, sh in res[:top]:
        ms = time_of(sh)
        log(f"  {ms:.4f} ms  {sh}")
        again.append((ms, sh))
    return min(again, key=lambda r: r[0])


def tune_eig3(P, dtype, label, shapes, taus, extra, log, top=3, aos=False, limits=None):
    n = P.shape[1]
    kw = dict(dtype=P.dtype, device=P.device)
    out = {"lam": torch.empty((3, n), **kw), "D": torch.empty((9, n), **kw), "phi": torch.empty((3, n), **kw)}
    X = P.T.contiguous() if aos else P

    def run(o):
        if aos:
            ksym.eig3_aos(X, opts=o, out=out)
        else:
            ksym.eig3(X, opts=o, out=out)

    log(f"[{label}] stage 1: {len(shapes)} launch shapes")
    res = _sweep(run, dtype, shapes, extra, log)
    # stage 2: the largest threshold that meets the accuracy limits on the
    # fastest shape (a larger tau_res refines fewer matrices; the results of
    # a threshold do not depend on the launch shape)
    sh0 = res[0][1]
    log(f"[{label}] stage 2: thresholds {taus} on {sh0}")
    tau_ok, acc_ok = None, None
    for tau in sorted(taus):
        run(ksym.Opts.defaults(dtype, **sh0, **extra, tau_res=tau))
        torch.cuda.synchronize()
        acc = _accuracy3(P, out)
        ok = _ok(acc, limits)
        log(f"  tau_res {tau:g} ok={ok} {acc}")
        if ok:
            tau_ok, acc_ok = tau, acc
    if tau_ok is None:
        raise RuntimeError(f"{label}: no setting met the accuracy targets")
    # stage 3: the fastest shapes timed again at that threshold
    log(f"[{label}] stage 3: the {top} fastest shapes at tau_res {tau_ok:g}")
    best = None
    for ms0, sh in res[:top]:
        o = ksym.Opts.defaults(dtype, **sh, **extra, tau_res=tau_ok)
        ms = _time(lambda: run(o))
        log(f"  {ms:.4f} ms {sh}")
        if best is None or ms < best["ms"]:
            best = {"ms": ms, "opts": dict(sh, **extra, tau_res=tau_ok), "accuracy": acc_ok}
    ws = ksym.workspace()
    o = ksym.Opts.defaults(dtype, **best["opts"])
    if aos:
        ksym.eig3_aos(X, opts=o, out=out, ws=ws)
    else:
        ksym.eig3(X, opts=o, out=out, ws=ws)
    torch.cuda.synchronize()
    best["refined_fraction"] = int(ws[0].item()) / n
    best["n"] = n
    return best


def tune_mixed(log, shapes):
    import synth
    total = 1 << 26
    sizes, kinds = synth.mixed_group_sizes(total)
    rng = np.random.default_rng(synth.BASE_SEED + 1002)
    groups = []
    for s, k in zip(sizes, kinds):
        s = int(s)
        # every plane on a 256-byte boundary (the streaming kernel variant)
        P = rng.standard_normal((6 if k == 3 else 3, s), dtype=np.float32)
        planes = ksym.line_aligned_planes(P.shape[0], s, fill=P)
        if k == 3:
            out = {"lam": ksym.line_aligned_planes(3, s), "D": ksym.line_aligned_planes(9, s),
                   "phi": ksym.line_aligned_planes(3, s)}
        else:
            out = {"lam": ksym.line_aligned_planes(2, s), "D": ksym.line_aligned_planes(4, s),
                   "phi": ksym.line_aligned_planes(1, s)[0]}
        groups.append((int(k), planes, out))
    log(f"[mixed/f32] {len(shapes)} launch shapes, {total} matrices in {len(groups)} groups")
    stream = torch.cuda.Stream()

    def time_of(sh):
        plan = ksym.Plan(groups, opts=ksym.Opts.defaults(ksym.F32, **sh))
        with torch.cuda.stream(stream):
            plan.capture(stream)
        torch.cuda.synchronize()
        cur = torch.cuda.current_stream()
        ms = _time(lambda: plan.replay(cur))
        plan.close()
        return ms

    res = []
    for sh in shapes:
        try:
            ms = time_of(sh)
        except ksym.KsymError as e:
            log(f"  skip {sh}: {e}")
            continue
        log(f"  {ms:.4f} ms  {sh}")
        res.append((ms, sh))
    res.sort(key=lambda r: r[0])
    ms, sh = _retime_top(res, time_of, log)
    return {"ms": ms, "opts": dict(sh), "n": total}


def tune_eig2(log, shapes):
    import synth
    n = 1 << 24
    P = torch.from_numpy(synth.make_plain(16, n, dtype=np.float32)["planes2"]).cuda()
    out = {"lam": torch.empty((2, n), device="cuda"), "D": torch.empty((4, n), device="cuda"),
           "phi": torch.empty((n,), device="cuda"), "flags": None}
    log(f"[eig2/f32] {len(shapes)} launch shapes")
    res = _sweep(lambda o: ksym.eig2(P, opts=o, out=out), ksym.F32, shapes, {}, log)
    ms, sh = _retime_top(res, lambda sh: _time(lambda: ksym.eig2(P, opts=ksym.Opts.defaults(ksym.F32, **sh),
                                                                 out=out)), log)
    return {"ms": ms, "opts": dict(sh), "n": n}


def tune_eig3_lam(log, shapes):
    """The eigenvalues-only mode (float32, no D and no angle planes): launch
    shapes only (it has no refinement thresholds); the eigenvalues are checked
    against LAPACK on a sample."""
    import synth
    n = 1 << 24
    P = torch.from_numpy(synth.make_precision(n)).cuda()
    out = {"lam": torch.empty((3, n), device="cuda")}
    log(f"[eig3_lam/f32] {len(shapes)} launch shapes")
    res = _sweep(lambda o: ksym.eig3(P, opts=o, out=out), ksym.F32, shapes, {}, log)
    ms, sh = _retime_top(res, lambda sh: _time(lambda: ksym.eig3(P, opts=ksym.Opts.defaults(ksym.F32, **sh),
                                                                 out=out)), log)
    ksym.eig3(P, opts=ksym.Opts.defaults(ksym.F32, **sh), out=out)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    idx = torch.from_numpy(np.sort(rng.choice(n, size=1 << 15, replace=False))).cuda()
    a11, a22, a33, a12, a13, a23 = P[:, idx].double().cpu().numpy()
    A = np.stack([np.stack([a11, a12, a13], 1), np.stack([a12, a22, a23], 1), np.stack([a13, a23, a33], 1)], 1)
    lam = np.sort(out["lam"][:, idx].double().cpu().numpy().T, axis=1)
    fro = np.sqrt((A * A).sum((1, 2)))
    err = float((np.abs(lam - np.linalg.eigvalsh(A)).max(1) / np.where(fro > 0, fro, 1)).max())
    if not err <= LAM_TOL:
        raise RuntimeError(f"eig3_lam/f32: eigenvalue error {err:g} above {LAM_TOL:g}")
    return {"ms": ms, "opts": dict(sh), "n": n, "accuracy": {"lam_err_max": err}}


def main(argv=None):
    ap = argparse.ArgumentParser(description="ksym autotuner (writes tuned.json)")
    ap.add_argument("--kinds", default="eig3/f32,eig3_grad/f32,eig3_aos/f32,eig3/f64,mixed/f32,eig2/f32,"
                                       "eig3_lam/f32")
    ap.add_argument("--quick", action="store_true", help="a smaller search space")
    ap.add_argument("--out", default=os.path.join(HERE, "tuned.json"))
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("the autotuner needs a GPU")
    import synth

    def log(msg):
        print(msg, flush=True)

    kinds = args.kinds.split(",")
    tuned = {}
    if os.path.exists(args.out):
        with open(args.out) as f:
            tuned = json.load(f)
    # large grid_mult values make the launch non-persistent (one wave tile
    # per wave), which measured fastest for the 3x3 kernels
    gms = (16, 64, 256, 65536) if args.quick else (4, 16, 32, 64, 128, 256, 512, 1024, 65536)
    drains = (0, 8) if args.quick else (0, 4, 8, 16)
    shapes32 = _shapes((64, 128, 256, 512), (1, 2), gms, drains)
    shapes_aos = [s for s in shapes32 if (s["block"], s["mats_per_lane"]) in
                  ((64, 1), (128, 1), (256, 1), (256, 2), (512, 1))]
    shapes64 = [s for s in _shapes((64, 128, 256), (1, 2), gms, drains)
                if s["mats_per_lane"] == 1 or s["block"] == 256]
    dev = torch.cuda.get_device_name(0)
    t0 = time.time()
    for kind in kinds:
        if kind == "eig3/f32":
            P = torch.from_numpy(synth.make_precision(1 << 24)).cuda()
            rec = tune_eig3(P, ksym.F32, kind, shapes32, (1e-6, 2e-6, 3e-6, 4e-6), {}, log)
            rec["workload"] = "precision recipe, 2^24 float32, SoA"
        elif kind == "eig3_grad/f32":
            d = synth.make_grad(1 << 22)
            P = torch.from_numpy(d["planes3"]).cuda()
            rec = tune_eig3(P, ksym.F32, kind, shapes32, (2e-6,), {"tau_vec": 1e-4}, log)
            rec["workload"] = "gradient recipe, 2^22 float32, N(0,1), relative gap >= 1e-3, tau_vec 1e-4"
        elif kind == "eig3_aos/f32":
            f = synth.make_field(256, 256, 256)
            P = torch.from_numpy(np.ascontiguousarray(f["aos"].T)).cuda()
            rec = tune_eig3(P, ksym.F32, kind, shapes_aos, (1e-6, 2e-6, 3e-6), {"tau_vec": 1e-4}, log, aos=True)
            rec["workload"] = "256^3 SPD tensor field, AoS float32, tau_vec 1e-4"
        elif kind == "eig3/f64":
            P = torch.from_numpy(synth.make_precision(1 << 24)).cuda().double()
            rec = tune_eig3(P, ksym.F64, kind, shapes64, (1e-11,), {"path": ksym.PATH_FP64_FIXUP}, log, top=1,
                            limits=LIMITS_F64)
            rec["workload"] = "precision recipe promoted to float64, checked path"
        elif kind == "mixed/f32":
            rec = tune_mixed(log, [s for s in shapes32 if (s["block"], s["mats_per_lane"]) in
                                   ((64, 1), (128, 1), (256, 1), (256, 2), (512, 1))])
            rec["workload"] = "2^26 mixed 2x2/3x3 in 1024 groups, planes 256-byte aligned, graph replay"
        elif kind == "eig2/f32":
            rec = tune_eig2(log, _shapes((64, 128, 256, 512, 1024), (1, 2, 4), gms, (0,)))
            rec["workload"] = "2^24 float32 2x2, U[-1,1]"
        elif kind == "eig3_lam/f32":
            rec = tune_eig3_lam(log, _shapes((64, 128, 256, 512), (1, 2), gms, (0,)))
            rec["workload"] = "precision recipe, 2^24 float32, SoA, eigenvalues only"
        else:
            raise SystemExit(f"unknown kind {kind}")
        rec["device"] = dev
        rec["library_version"] = ksym.version()
        tuned[kind] = rec
        log(f"[{kind}] chose {rec['opts']} at {rec['ms']:.4f} ms")
        with open(args.out, "w") as f:
            json.dump(tuned, f, indent=1, sort_keys=True)
        torch.cuda.empty_cache()
    log(f"done in {time.time() - t0:.0f} s -> {args.out}")


if __name__ == "__main__":
    main()
