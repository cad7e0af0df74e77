"""Benchmark of the MF-WQ hot path on one MI355X.

Workload: the thick quarter ring (spline geometry + 0.02 smooth noise, K = I,
oscillating source), 64 elements per direction, degrees p = 2..6 -- the
full-size FP64 configuration of the benchmark (degrees 3..6, plus p = 2 that the
metric also names).  Inputs are synthetic and seeded (``synth``).

One step = for every degree p:
  * FP64 operator applies w = K~ v on the stream the library runs on: R with
    HIP events around each, R back to back between two events, and R
    accumulating applies (no clearing of w) back to back,
  * one FP64 right-preconditioned BiCGStab solve to relative residual 1e-10,
  * one mixed-precision solve (FP32 apply, FP32 FD by default, FP64 refinement)
    to the same residual,
  * the adjoint of J = 1/2 |u|^2 at the FP64 solution: transposed solve
    K~^T lam = u to 1e-10, then dJ/dC (six planes) and dJ/df at every
    quadrature point, and R/4 timed transposed applies.
Set-up (splines, weights, geometry, FD eigenpairs) is outside the timed region.

value   = FP64 apply throughput, sum_p N_p * applies / sum of apply times (GDOF/s);
          an apply is the clearing of w plus the fused kernel (wq_apply), timed
          as R applies back to back between two HIP events; the same applies
          are also timed one launch at a time (events around each launch, which
          adds the events' own cost) for the p10/p90 spread
roofline: algorithmic bytes of one FP64 apply = 48 N_q + 16 N (six coefficient
          planes read once, v read and w written once) over the average duration
          of the fused kernel alone: R back-to-back accumulating applies
          (wq_apply_acc, which skips the clearing) between two HIP events.
          traffic: DRAM-side bytes per launch from the committed counter summary
          in profiles/ (FETCH_SIZE + WRITE_SIZE scaled by a copy of known size),
          reported only while the kernel source still matches the hash recorded
          there.
Equal accuracy: besides the runs to relative residual 1e-10, each degree is also
solved at the loosest residual tolerance whose solution is within 1e-10
(relative 2-norm) of a tight reference solve (FP64, residual 1e-13), for both
the FP64 and the mixed solver; those times are the like-for-like comparison.
roofline_fd: the FD preconditioner (three fused mode-product passes) timed
          alone, R back-to-back FP64 applications between two HIP events per
          degree; algorithmic flops 12 n N + N per application (six mode products
          of 2 n N flops and the diagonal scaling) over FP64 MFMA peak.  FP32 and
          BF16 times are reported per degree against their own peaks.
Statistics: p10/p90 of the per-launch apply times; "flushed": the fused
          kernel timed launch by launch right after a 512 MiB write that evicts
          the 256 MB last-level cache (the C2 coefficient set fits in it).
large_workloads: after the timed steps, ring 96^3 p = 5 and the twisted cube
          128^3 p = 6 with full anisotropic K (coefficient sets of 0.4 and 0.9 GB
          FP64, larger than the last-level cache): kernel-alone FP64 and FP32
          applies (warm and flushed), FD times, one FP64 and one mixed solve.
cpu_baseline: the CPU FP64 oracle on this host within a bounded budget:
          value = its matrix-free apply on degree 3 of the same workload with
          all threads; also single-threaded (the paper's setting) and FD-
          preconditioned BiCGStab solves to 1e-10 on the identity cube (12^3,
          p = 3), the ring (64^3, p = 3) and the log-normal kappa ring (48^3,
          p = 4).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import re
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}    # dense, MI355X
METRIC = "WQ apply GDOF/s & time-to-solve to rel.res 1e-10, FP64 vs mixed, p=2..6"


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "wq_apply_fused_f64_ring64_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1712_08565_amd", "csrc", f) for f in ("wq_fused.hip", "fused.h", "buffer.h")]
EQ_TOL = 1e-10
RTOL_LADDER = [1e-10, 3e-11, 1e-11, 3e-12, 1e-12, 3e-13, 1e-13]


def _code_only(text: str) -> str:
    """The source without comments, trailing blanks and empty lines (the kernel
    sources hold no string literals with comment markers)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip())


def kernel_hash() -> str:
    """sha256 of the code of the fused-apply sources (comments excluded, so that
    a counter summary stays valid across comment edits)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()


def committed_traffic(degrees, reaction=False):
    """Mean DRAM-side bytes per FP64 apply over ``degrees`` from the counter
    summary (the kernels with the reaction term when ``reaction``), or None if
    it is missing, stale (kernel source changed) or lacks a degree."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    sha, per_p = None, {}
    for ln in lines:
        if ln.startswith("# kernel sha256:"):
            sha = ln.split(":", 1)[1].strip()
        elif ln.startswith("reaction p=" if reaction else "p=") and "traffic_bytes=" in ln:
            kv = dict(t.split("=", 1) for t in ln.split() if "=" in t)
            per_p[int(kv["p"])] = float(kv["traffic_bytes"])
    if sha != kernel_hash() or any(p not in per_p for p in degrees):
        return None
    return sum(per_p[p] for p in degrees) / len(degrees)


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def grad_bytes(A):
    """Algorithmic bytes of one wq_grad_Kf: dJ/dK (six planes for identity or
    six-component K, one for scalar K) and dJ/df written, det J read (and the nine
    planes of J^{-1} for the chain of a scalar or six-component K), lam and u read."""
    from paper_1712_08565_amd.wqfd import WQ_K_IDENTITY, WQ_K_SCALAR
    out = 1 if A.k_kind == WQ_K_SCALAR else 6
    geo = 1 if A.k_kind == WQ_K_IDENTITY else 10
    return 8 * A.Nq * (out + 1 + geo) + 16 * A.N


def cpu_baseline(budget_s: float, solve_budget_s: float = 25.0):
    """The CPU FP64 oracle on this host: matrix-free apply on ring64 p=3 with all
    threads (value) and with one, and FD-preconditioned BiCGStab solves to 1e-10
    on the identity cube, the ring and the log-normal kappa ring (each with a
    bounded iteration count when the budget runs out)."""
    import numpy as np

    import synth
    from oracle.fd import FD
    from oracle.krylov import bicgstab
    from oracle.operator import Problem
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threadpool_limits = None
        threads = os.cpu_count()
    wl = synth.workload("ring64_p3")
    t0 = time.perf_counter()
    pr = Problem(wl.knots(), wl.p, wl.ctrl(), wl.K_field())
    log(f"cpu oracle setup {time.perf_counter() - t0:.1f}s")
    v = synth.random_vector(pr.N, 42)
    pr.apply(v)  # warm-up

    def timed(budget, cap):
        times = []
        t_start = time.perf_counter()
        while True:
            t0 = time.perf_counter()
            pr.apply(v)
            times.append(time.perf_counter() - t0)
            if time.perf_counter() - t_start > budget or len(times) >= cap:
                return float(np.median(times)), len(times)

    t, n_all = timed(0.4 * budget_s, 100)
    out = {"value": pr.N / t / 1e9, "unit": "GDOF/s", "cores": int(threads), "kind": "oracle",
           "sample": f"ring64 p=3 (N={pr.N}), {n_all} FP64 matrix-free applies, median {t:.3f} s each; "
                     f"host cpus={os.cpu_count()}, affinity={len(os.sched_getaffinity(0))}"}
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            t1, n1 = timed(0.15 * budget_s, 20)
        out["single_thread"] = {"value": pr.N / t1 / 1e9, "unit": "GDOF/s", "cores": 1,
                                "sample": f"ring64 p=3, {n1} applies, median {t1:.3f} s"}
    if solve_budget_s > 0:
        res = {}
        for name in ("cube12_p3", "ring64_p3", "ring48_p4_kappa"):
            w = synth.workload(name)
            q = pr if name == "ring64_p3" else Problem(w.knots(), w.p, w.ctrl(), w.K_field())
            fd = FD(q.spaces)
            b = q.rhs_from(w.f())
            # per-iteration cost from one apply + FD, then an iteration cap within the budget
            t0 = time.perf_counter()
            fd.apply(q.apply(b))
            it_cost = 2 * (time.perf_counter() - t0)
            cap = max(1, int(solve_budget_s / max(it_cost, 1e-6)))
            t0 = time.perf_counter()
            _, it, rel, _ = bicgstab(q.apply, b, fd.apply, tol=1e-10, maxit=cap)
            ts = time.perf_counter() - t0
            res[name] = {"N": q.N, "seconds": round(ts, 3), "iters": int(it), "relres": float(rel),
                         "converged": bool(rel <= 1e-10)}
            log(f"cpu oracle solve {name}: {it} it, {ts:.1f}s, relres {rel:.1e}")
        out["solves_rtol_1e-10"] = res
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--degrees", default="2,3,4,5,6")
    ap.add_argument("--n-el", type=int, default=64)
    ap.add_argument("--reps", type=int, default=20, help="timed applies per degree per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds for the oracle's apply timings")
    ap.add_argument("--cpu-solve-budget", type=float, default=25.0,
                    help="seconds per oracle solve (iteration cap from the measured iteration cost; 0: skip)")
    ap.add_argument("--no-solve", action="store_true", help="time the applies only")
    ap.add_argument("--workloads", default="",
                    help="comma-separated named workloads instead of the default ring (e.g. ring96_p5,twist128_p6)")
    ap.add_argument("--mixed-fd", choices=("f32", "bf16"), default="f32", help="FD precision of the inner solves")
    ap.add_argument("--mixed-tau", type=float, default=1e-4, help="inner relative tolerance of the refinement")
    ap.add_argument("--reaction-degree", type=int, default=3,
                    help="degree of the reaction-term measurement on the same ring (0: skip)")
    ap.add_argument("--gauss-degrees", default="",
                    help="degrees of a Gauss-quadrature comparison on the same ring (e.g. 2,3,4; off by default: "
                         "it launches the same kernel instances as the timed applies)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the out-of-cache records (ring 96^3 p = 5, twisted cube 128^3 p = 6)")
    ap.add_argument("--flush-mib", type=int, default=512,
                    help="size of the cache-evicting write before each flushed-kernel launch (0: skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one device copy of this many MiB per step (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the multi-GPU (z-slab) decomposition is a design note, "
              "not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1712_08565_amd import problem, wqfd

    torch.cuda.set_device(0)
    MIX_FD = wqfd.WQ_F32 if args.mixed_fd == "f32" else wqfd.WQ_BF16
    MIX_TAU = args.mixed_tau

    def solve(P, kind, rtol, x=None):
        dp = P["dp"]
        x = torch.zeros_like(P["v"]) if x is None else x.zero_()
        if kind == "fp64":
            _, it, res = wqfd.krylov_solve(dp.A, dp.P, dp.b, x=x, rtol=rtol, maxit=2000, ws=P["kws"])
            P["last"] = (it, 0, res)
        else:
            _, outer, inner, res = wqfd.ir_solve(dp.A, dp.P, dp.b, x=x, fd_prec=MIX_FD, rtol=rtol,
                                                 tau_inner=MIX_TAU, ws=P["iws"])
            P["last"] = (outer, inner, res)
        return x

    degrees = [int(x) for x in args.degrees.split(",")]
    if args.workloads:                       # named workloads (other full-size configurations)
        cases = [(name, synth.workload(name)) for name in args.workloads.split(",")]
    else:
        cases = [(f"p{p}", synth.Workload(f"ring{args.n_el}_p{p}", args.n_el, p, "ring", 0.02, "identity", "paper"))
                 for p in degrees]
    keys = [k for k, _ in cases]
    probs = {}
    for p, wl in cases:
        t0 = time.perf_counter()
        dp = problem.build(wl, wqfd.WQ_F64 | wqfd.WQ_F32, wqfd.WQ_F64 | wqfd.WQ_F32 | wqfd.WQ_BF16)
        torch.cuda.synchronize()
        v = torch.as_tensor(synth.random_vector(dp.A.N, 42), device="cuda")
        w = torch.empty_like(v)
        kws = torch.empty(wqfd.lib().krylov_ws_bytes(dp.A.handle), dtype=torch.uint8, device="cuda")
        iws = torch.empty(wqfd.lib().ir_ws_bytes(dp.A.handle), dtype=torch.uint8, device="cuda")
        # reference solution for the equal-accuracy comparison (outside the timed region)
        xref, it_ref, res_ref = None, 0, float("nan")
        if not args.no_solve:
            xref, it_ref, res_ref = wqfd.krylov_solve(dp.A, dp.P, dp.b, rtol=1e-13, maxit=2000, ws=kws,
                                                      raise_on_noconv=False)
        probs[p] = dict(dp=dp, v=v, w=w, wacc=torch.zeros_like(v), kws=kws, iws=iws, xref=xref, x=torch.zeros_like(v),
                        N=dp.A.N, Nq=dp.A.Nq, n=dp.A.n, setup_s=time.perf_counter() - t0,
                        v32=v.float(), z32=torch.empty(dp.A.N, dtype=torch.float32, device="cuda"))
        if not args.no_solve:
            planes = 1 if dp.A.k_kind == wqfd.WQ_K_SCALAR else 6
            probs[p].update(lam=torch.zeros_like(v),
                            gK=torch.empty(planes * dp.A.Nq, dtype=torch.float64, device="cuda"),
                            gf=torch.empty(dp.A.Nq, dtype=torch.float64, device="cuda"))
        if not args.no_solve:
            nref = torch.linalg.norm(xref).item()
            P = probs[p]
            for kind in ("fp64", "mixed"):
                P[f"{kind}_eq_rtol"] = None
                # the loosest tolerance that meets the accuracy twice in a row with a
                # factor-2 margin (the applies accumulate with atomics, so repeated
                # solves differ in the last bits and the final error varies)
                for rt in RTOL_LADDER:
                    try:
                        errs = [torch.linalg.norm(solve(P, kind, rt) - xref).item() / nref for _ in range(2)]
                    except RuntimeError as e:          # no convergence at this tolerance
                        log(f"p={p} {kind} rtol {rt:.0e}: {e}")
                        continue
                    if max(errs) <= EQ_TOL / 2:
                        P[f"{kind}_eq_rtol"] = rt
                        break
        log(f"setup p={p}: N={dp.A.N} Nq={dp.A.Nq} {probs[p]['setup_s']:.1f}s (ref solve {it_ref} it, "
            f"relres {res_ref:.1e}); equal-accuracy rtol fp64 {probs[p].get('fp64_eq_rtol')} "
            f"mixed {probs[p].get('mixed_eq_rtol')}")

    stream = torch.cuda.current_stream()
    rec = {p: dict(apply_ms=[], launch_ms=[], kernel_ms=[], fd_ms={"f64": [], "f32": [], "bf16": []}, fp64_ms=[], fp64_it=[], fp64_err=[], mix_ms=[], mix_outer=[], mix_inner=[],
                   mix_err=[], fp64_eq_ms=[], fp64_eq_err=[], fp64_eq_it=[], mixed_eq_ms=[], mixed_eq_err=[],
                   mixed_eq_it=[], adj_ms=[], adj_it=[], grad_ms=[], applyT_ms=[]) for p in keys}
    probe = None
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 8
        probe = (torch.ones(n, dtype=torch.float64, device="cuda"), torch.empty(n, dtype=torch.float64, device="cuda"))

    def one_step(record: bool):
        for p in keys:
            P = probs[p]
            dp = P["dp"]
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(args.reps)]
            for e0, e1 in evs:
                e0.record(stream)
                wqfd.wq_apply(dp.A, P["v"], P["w"])
                e1.record(stream)
            b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            b0.record(stream)
            for _ in range(args.reps):
                wqfd.wq_apply(dp.A, P["v"], P["w"])
            b1.record(stream)
            k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            k0.record(stream)
            for _ in range(args.reps):
                wqfd.wq_apply_acc(dp.A, P["v"], P["wacc"])
            k1.record(stream)
            fd_ev = {}
            for fname, fprec, r_, z_ in (("f64", wqfd.WQ_F64, P["v"], P["w"]), ("f32", wqfd.WQ_F32, P["v32"], P["z32"]),
                                         ("bf16", wqfd.WQ_BF16, P["v32"], P["z32"])):
                f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                f0.record(stream)
                for _ in range(args.reps):
                    wqfd.fd_apply(dp.P, r_, z_, prec=fprec)
                f1.record(stream)
                fd_ev[fname] = (f0, f1)
            if not args.no_solve:
                P["x"].zero_()
                s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                s0.record(stream)
                _, it, res = wqfd.krylov_solve(dp.A, dp.P, dp.b, x=P["x"], rtol=1e-10, maxit=2000, ws=P["kws"])
                s1.record(stream)
                xm = torch.zeros_like(P["x"])
                m0, m1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                m0.record(stream)
                _, outer, inner, mres = wqfd.ir_solve(dp.A, dp.P, dp.b, x=xm, fd_prec=MIX_FD, rtol=1e-10,
                                                      tau_inner=MIX_TAU, ws=P["iws"])
                m1.record(stream)
                eq = {}
                for kind in ("fp64", "mixed"):
                    rt = P[f"{kind}_eq_rtol"]
                    if rt is None:
                        continue
                    q0, q1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    xq = torch.zeros_like(P["x"])
                    q0.record(stream)
                    solve(P, kind, rt, xq)
                    q1.record(stream)
                    eq[kind] = (q0, q1, xq, P["last"])
                # adjoint of J = 1/2 |u|^2 at the FP64 solution (transposed solve + gradient kernels)
                a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                P["lam"].zero_()
                a0.record(stream)
                _, ait, _ = wqfd.krylov_solve(dp.A, dp.P, P["x"], x=P["lam"], transpose=True, rtol=1e-10,
                                              maxit=2000, ws=P["kws"])
                wqfd.wq_grad_Kf(dp.A, P["lam"], P["x"], P["gK"], P["gf"])
                a1.record(stream)
                # the gradient kernels alone (dJ/dK and dJ/df at the adjoint state)
                g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                g0.record(stream)
                for _ in range(max(1, args.reps // 4)):
                    wqfd.wq_grad_Kf(dp.A, P["lam"], P["x"], P["gK"], P["gf"])
                g1.record(stream)
                evT = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                       for _ in range(max(1, args.reps // 4))]
                for e0, e1 in evT:
                    e0.record(stream)
                    wqfd.wq_apply_T(dp.A, P["v"], P["w"])
                    e1.record(stream)
            if probe is not None:
                probe[1].copy_(probe[0])
            torch.cuda.synchronize()
            if record:
                r = rec[p]
                r["launch_ms"] += [e0.elapsed_time(e1) for e0, e1 in evs]
                r["apply_ms"] += [b0.elapsed_time(b1) / args.reps] * args.reps
                r["kernel_ms"] += [k0.elapsed_time(k1) / args.reps] * args.reps
                for fname, (f0, f1) in fd_ev.items():
                    r["fd_ms"][fname].append(f0.elapsed_time(f1) / args.reps)
                if not args.no_solve:
                    nref = torch.linalg.norm(P["xref"]).item()
                    r["fp64_ms"].append(s0.elapsed_time(s1))
                    r["fp64_it"].append(it)
                    r["fp64_err"].append(torch.linalg.norm(P["x"] - P["xref"]).item() / nref)
                    r["mix_ms"].append(m0.elapsed_time(m1))
                    r["mix_outer"].append(outer)
                    r["mix_inner"].append(inner)
                    r["mix_err"].append(torch.linalg.norm(xm - P["xref"]).item() / nref)
                    r["adj_ms"].append(a0.elapsed_time(a1))
                    r["adj_it"].append(ait)
                    r["grad_ms"].append(g0.elapsed_time(g1) / max(1, args.reps // 4))
                    r["applyT_ms"] += [e0.elapsed_time(e1) for e0, e1 in evT]
                    for kind, (q0, q1, xq, last) in eq.items():
                        r[f"{kind}_eq_ms"].append(q0.elapsed_time(q1))
                        r[f"{kind}_eq_err"].append(torch.linalg.norm(xq - P["xref"]).item() / nref)
                        r[f"{kind}_eq_it"].append(last[0] if kind == "fp64" else last[1])

    # reaction term alpha u (mass apply of Algorithm 1 inside the fused kernels):
    # its own operator on the ring, alpha = 10 n_el^2 (1 + ...) so that M~ and K~
    # are of the same size, FD shifted by mean(alpha det J)
    react = None
    if args.reaction_degree and not args.workloads:
        rp = args.reaction_degree
        wl = synth.Workload(f"ring{args.n_el}_p{rp}", args.n_el, rp, "ring", 0.02, "identity", "paper")
        dpr = problem.build(wl, wqfd.WQ_F64 | wqfd.WQ_F32, wqfd.WQ_F64 | wqfd.WQ_F32 | wqfd.WQ_BF16)
        _, sigma = problem.set_reaction(dpr, synth.alpha_field(10.0 * args.n_el ** 2))
        vr = torch.as_tensor(synth.random_vector(dpr.A.N, 42), device="cuda")
        react = dict(dp=dpr, v=vr, w=torch.empty_like(vr), wacc=torch.zeros_like(vr), x=torch.zeros_like(vr),
                     kws=torch.empty(wqfd.lib().krylov_ws_bytes(dpr.A.handle), dtype=torch.uint8, device="cuda"),
                     iws=torch.empty(wqfd.lib().ir_ws_bytes(dpr.A.handle), dtype=torch.uint8, device="cuda"),
                     sigma=sigma, apply_ms=[], kernel_ms=[], fp64_ms=[], fp64_it=[], mix_ms=[], mix_inner=[])
        torch.cuda.synchronize()

    def reaction_step(record: bool):
        R = react
        dpr = R["dp"]
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.reps)]
        for e0, e1 in evs:
            e0.record(stream)
            wqfd.wq_apply(dpr.A, R["v"], R["w"])
            e1.record(stream)
        k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        k0.record(stream)
        for _ in range(args.reps):
            wqfd.wq_apply_acc(dpr.A, R["v"], R["wacc"])
        k1.record(stream)
        if not args.no_solve:
            R["x"].zero_()
            s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s0.record(stream)
            _, it, _ = wqfd.krylov_solve(dpr.A, dpr.P, dpr.b, x=R["x"], rtol=1e-10, maxit=2000, ws=R["kws"])
            s1.record(stream)
            xm = torch.zeros_like(R["x"])
            m0, m1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            m0.record(stream)
            _, _, inner, _ = wqfd.ir_solve(dpr.A, dpr.P, dpr.b, x=xm, fd_prec=MIX_FD, rtol=1e-10, tau_inner=MIX_TAU,
                                           ws=R["iws"])
            m1.record(stream)
        torch.cuda.synchronize()
        if record:
            R["apply_ms"] += [e0.elapsed_time(e1) for e0, e1 in evs]
            R["kernel_ms"].append(k0.elapsed_time(k1) / args.reps)
            if not args.no_solve:
                R["fp64_ms"].append(s0.elapsed_time(s1))
                R["fp64_it"].append(it)
                R["mix_ms"].append(m0.elapsed_time(m1))
                R["mix_inner"].append(inner)

    for i in range(args.warmup):
        one_step(False)
        log(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        one_step(True)
        log(f"step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # after the timed steps (not part of them): the fused kernel launch by launch
    # right after a write that evicts the last-level cache
    flush = None
    if args.flush_mib > 0:
        flush = torch.empty((args.flush_mib << 20) // 4, dtype=torch.float32, device="cuda")

    def flushed_kernel_ms(A, v, wacc, prec, reps):
        out = []
        for i in range(reps):
            flush.fill_(float(i))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            wqfd.wq_apply_acc(A, v, wacc, prec=prec)
            e1.record(stream)
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        return out

    flushed = {}
    if flush is not None:
        for p in keys:
            P = probs[p]
            flushed[p] = flushed_kernel_ms(P["dp"].A, P["v"], P["wacc"], wqfd.WQ_F64, args.reps)
        log("flushed-cache kernel timings done")

    def fd_times(dp, v64, v32, reps):
        z64, z32 = torch.empty_like(v64), torch.empty_like(v32)
        t = {}
        for fname, fprec, r_, z_ in (("f64", wqfd.WQ_F64, v64, z64), ("f32", wqfd.WQ_F32, v32, z32),
                                     ("bf16", wqfd.WQ_BF16, v32, z32)):
            wqfd.fd_apply(dp.P, r_, z_, prec=fprec)
            f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            f0.record(stream)
            for _ in range(reps):
                wqfd.fd_apply(dp.P, r_, z_, prec=fprec)
            f1.record(stream)
            torch.cuda.synchronize()
            t[fname] = f0.elapsed_time(f1) / reps
        return t

    # out-of-cache workloads: ring 96^3 p = 5 and the twisted cube 128^3 p = 6
    large = {}
    if not args.no_large and not args.workloads:
        for name in ("ring96_p5", "twist128_p6"):
            wl = synth.workload(name)
            t0l = time.perf_counter()
            dpl = problem.build(wl, wqfd.WQ_F64 | wqfd.WQ_F32, wqfd.WQ_F64 | wqfd.WQ_F32 | wqfd.WQ_BF16)
            torch.cuda.synchronize()
            setup_l = time.perf_counter() - t0l
            A = dpl.A
            vl = torch.as_tensor(synth.random_vector(A.N, 42), device="cuda")
            vl32 = vl.float()
            acc64, acc32 = torch.zeros_like(vl), torch.zeros_like(vl32)
            rec_l = {}
            for prec, vv, acc, key in ((wqfd.WQ_F64, vl, acc64, "f64"), (wqfd.WQ_F32, vl32, acc32, "f32")):
                wqfd.wq_apply_acc(A, vv, acc, prec=prec)
                k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                k0.record(stream)
                for _ in range(args.reps):
                    wqfd.wq_apply_acc(A, vv, acc, prec=prec)
                k1.record(stream)
                torch.cuda.synchronize()
                s_ = 8 if prec == wqfd.WQ_F64 else 4
                alg = 6 * s_ * A.Nq + 2 * s_ * A.N
                t_k = k0.elapsed_time(k1) / args.reps
                rec_l[f"kernel_{key}_ms"] = round(t_k, 4)
                rec_l[f"kernel_{key}_GBs"] = round(alg / t_k / 1e6, 1)
                rec_l[f"kernel_{key}_frac_of_hbm_peak"] = round(alg / t_k / 1e6 / HBM_PEAK_GBS, 4)
                rec_l[f"kernel_{key}_GDOFs"] = round(A.N / t_k / 1e6, 3)
                if flush is not None:
                    fl = flushed_kernel_ms(A, vv, acc, prec, max(5, args.reps // 2))
                    rec_l[f"kernel_{key}_flushed_ms_median"] = round(float(np.median(fl)), 4)
                    rec_l[f"kernel_{key}_flushed_frac_of_hbm_peak"] = round(
                        alg / float(np.median(fl)) / 1e6 / HBM_PEAK_GBS, 4)
            # adjoint gradient kernels (dJ/dK and dJ/df in one pass) at a random state
            lam_l = torch.as_tensor(synth.random_vector(A.N, 45), device="cuda")
            gK_l, gf_l = wqfd.wq_grad_Kf(A, lam_l, vl)
            g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            g0.record(stream)
            for _ in range(args.reps):
                wqfd.wq_grad_Kf(A, lam_l, vl, gK_l, gf_l)
            g1.record(stream)
            torch.cuda.synchronize()
            t_g = g0.elapsed_time(g1) / args.reps
            rec_l["gradient_kernels_ms"] = round(t_g, 4)
            rec_l["gradient_over_apply"] = round(t_g / rec_l["kernel_f64_ms"], 2)
            rec_l["gradient_GBs"] = round(grad_bytes(A) / t_g / 1e6, 1)
            rec_l["gradient_frac_of_hbm_peak"] = round(grad_bytes(A) / t_g / 1e6 / HBM_PEAK_GBS, 4)
            del lam_l, gK_l, gf_l
            ft = fd_times(dpl, vl, vl32, args.reps)
            nmax = max(A.n)
            fl_fd = 12 * nmax * A.N + A.N
            rec_l["fd_ms"] = {k: round(v_, 4) for k, v_ in ft.items()}
            rec_l["fd_frac_of_mfma_peak"] = {k: round(fl_fd / (v_ * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS[k], 4)
                                             for k, v_ in ft.items()}
            if not args.no_solve:
                kws = torch.empty(wqfd.lib().krylov_ws_bytes(A.handle), dtype=torch.uint8, device="cuda")
                iws = torch.empty(wqfd.lib().ir_ws_bytes(A.handle), dtype=torch.uint8, device="cuda")
                xl = torch.zeros_like(vl)
                s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                s0.record(stream)
                _, it, _ = wqfd.krylov_solve(A, dpl.P, dpl.b, x=xl, rtol=1e-10, maxit=2000, ws=kws)
                s1.record(stream)
                xm = torch.zeros_like(vl)
                m0, m1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                m0.record(stream)
                _, outer, inner, _ = wqfd.ir_solve(A, dpl.P, dpl.b, x=xm, fd_prec=wqfd.WQ_BF16, rtol=1e-10,
                                                   tau_inner=MIX_TAU, ws=iws)
                m1.record(stream)
                torch.cuda.synchronize()
                rec_l.update({"fp64_solve_ms": round(s0.elapsed_time(s1), 2), "fp64_iters": int(it),
                              "mixed_bf16_fd_solve_ms": round(m0.elapsed_time(m1), 2), "mixed_outer": int(outer),
                              "mixed_inner": int(inner),
                              "mixed_vs_fp64_rel_diff": torch.linalg.norm(xm - xl).item() / torch.linalg.norm(xl).item()})
            large[name] = dict(N=A.N, Nq=A.Nq, setup_s=round(setup_l, 2), **rec_l)
            del dpl, A, vl, vl32, acc64, acc32
            torch.cuda.empty_cache()
            log(f"large workload {name} done")
    if react is not None:                    # after the timed steps, not part of them
        for i in range(args.warmup + args.steps):
            reaction_step(i >= args.warmup)
        log("reaction-term measurement done")
    # Gauss-quadrature variant of the same operator (p + 1 Gauss points per element,
    # the same fused kernels): applies only, one operator at a time
    gauss = {}
    if args.gauss_degrees and not args.workloads:
        for gp in [int(x) for x in args.gauss_degrees.split(",")]:
            wl = synth.Workload(f"ring{args.n_el}_p{gp}", args.n_el, gp, "ring", 0.02, "identity", "paper")
            t0g = time.perf_counter()
            A = wqfd.wq_setup(gp, wl.knots(), wl.ctrl(), wqfd.WQ_K_IDENTITY, None, wqfd.WQ_F64, rule="gauss")
            setup_g = time.perf_counter() - t0g
            vg = torch.as_tensor(synth.random_vector(A.N, 42), device="cuda")
            wg, wgacc = torch.empty_like(vg), torch.zeros_like(vg)
            ap_ms, k_ms = [], []
            for i in range(args.warmup + args.steps):
                evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                       for _ in range(args.reps)]
                for e0, e1 in evs:
                    e0.record(stream)
                    wqfd.wq_apply(A, vg, wg)
                    e1.record(stream)
                k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                k0.record(stream)
                for _ in range(args.reps):
                    wqfd.wq_apply_acc(A, vg, wgacc)
                k1.record(stream)
                torch.cuda.synchronize()
                if i >= args.warmup:
                    ap_ms += [e0.elapsed_time(e1) for e0, e1 in evs]
                    k_ms.append(k0.elapsed_time(k1) / args.reps)
            gauss[gp] = dict(N=A.N, Nq=A.Nq, apply_ms=float(np.mean(ap_ms)), kernel_ms=float(np.mean(k_ms)),
                             setup_s=setup_g)
            del A, vg, wg, wgacc
            torch.cuda.empty_cache()
            log(f"gauss p={gp} done")

    tot_dof = sum(probs[p]["N"] * len(rec[p]["apply_ms"]) for p in keys)
    tot_s = sum(sum(rec[p]["apply_ms"]) for p in keys) / 1e3
    tot_bytes = sum((48 * probs[p]["Nq"] + 16 * probs[p]["N"]) * len(rec[p]["kernel_ms"]) for p in keys)
    tot_k = sum(sum(rec[p]["kernel_ms"]) for p in keys) / 1e3
    n_apply = sum(len(rec[p]["kernel_ms"]) for p in keys)
    achieved = tot_bytes / tot_k / 1e9
    traffic = None if args.workloads else committed_traffic(degrees)
    if traffic is not None:
        traffic = round(traffic)
    per_p = {}
    for p in keys:
        r = rec[p]
        t_ap = float(np.mean(r["apply_ms"]))
        d = {"N": probs[p]["N"], "Nq": probs[p]["Nq"], "apply_ms": round(t_ap, 4),
             "kernel_ms": round(float(np.mean(r["kernel_ms"])), 4),
             "apply_GDOFs": round(probs[p]["N"] / t_ap / 1e6, 3),
             "apply_GBs": round((48 * probs[p]["Nq"] + 16 * probs[p]["N"]) / t_ap / 1e6, 1),
             "apply_ms_one_launch": round(float(np.mean(r["launch_ms"])), 4),
             "apply_ms_one_launch_p10": round(float(np.percentile(r["launch_ms"], 10)), 4),
             "apply_ms_one_launch_p90": round(float(np.percentile(r["launch_ms"], 90)), 4),
             "setup_s": round(probs[p]["setup_s"], 2)}
        nmax = max(probs[p]["n"])
        fl_fd = 12 * nmax * probs[p]["N"] + probs[p]["N"]
        d["fd_ms"] = {k: round(float(np.mean(v_)), 4) for k, v_ in r["fd_ms"].items()}
        d["fd_frac_of_mfma_peak"] = {k: round(fl_fd / (float(np.mean(v_)) * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS[k], 4)
                                     for k, v_ in r["fd_ms"].items()}
        if p in flushed:
            t_fl = float(np.median(flushed[p]))
            d["kernel_flushed_ms_median"] = round(t_fl, 4)
            d["kernel_flushed_frac_of_hbm_peak"] = round((48 * probs[p]["Nq"] + 16 * probs[p]["N"]) / t_fl / 1e6
                                                         / HBM_PEAK_GBS, 4)
        if not args.no_solve:
            d.update({"fp64_solve_ms": round(float(np.median(r["fp64_ms"])), 2),
                      "fp64_iters": int(np.median(r["fp64_it"])),
                      "fp64_rel_err_vs_tight": float(np.max(r["fp64_err"])),
                      "mixed_solve_ms": round(float(np.median(r["mix_ms"])), 2),
                      "mixed_outer": int(np.median(r["mix_outer"])), "mixed_inner": int(np.median(r["mix_inner"])),
                      "mixed_rel_err_vs_tight": float(np.max(r["mix_err"]))})
            d["apply_T_ms"] = round(float(np.mean(r["applyT_ms"])), 4)
            d["adjoint_ms"] = round(float(np.median(r["adj_ms"])), 2)
            d["adjoint_iters"] = int(np.median(r["adj_it"]))
            d["gradient_kernels_ms"] = round(float(np.median(r["grad_ms"])), 4)
            d["gradient_over_apply"] = round(float(np.median(r["grad_ms"])) / t_ap, 2)
            gb = grad_bytes(probs[p]["dp"].A)
            d["gradient_GBs"] = round(gb / float(np.median(r["grad_ms"])) / 1e6, 1)
            d["gradient_frac_of_hbm_peak"] = round(gb / float(np.median(r["grad_ms"])) / 1e6 / HBM_PEAK_GBS, 4)
            for kind in ("fp64", "mixed"):
                if r[f"{kind}_eq_ms"]:
                    d[f"{kind}_equal_accuracy"] = {
                        "rtol": probs[p][f"{kind}_eq_rtol"], "ms": round(float(np.median(r[f"{kind}_eq_ms"])), 2),
                        "rel_err_vs_tight": float(np.max(r[f"{kind}_eq_err"])),
                        "iters": int(np.median(r[f"{kind}_eq_it"]))}
        per_p[p] = d
    out = {
        "metric": METRIC,
        "value": round(tot_dof / tot_s / 1e9, 4),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded spline ring geometry, K = I, oscillating source)",
        "config": {"workload": (f"thick quarter ring, {args.n_el}^3 elements, degrees {args.degrees}, "
                                f"FP64 apply + FP64 BiCGStab/FD and mixed-precision IR solves to rel.res 1e-10, "
                                f"adjoint gradient") if not args.workloads else
                   f"named workloads {args.workloads}: same step",
                   "n_el": args.n_el, "degrees": degrees if not args.workloads else None,
                   "workloads": keys, "applies_per_degree_per_step": args.reps,
                   "mixed": {"inner_fd": args.mixed_fd, "inner_apply": "f32", "tau_inner": args.mixed_tau}},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "wq_apply_fused_kernel<double, p, false> (timed alone via wq_apply_acc)",
                     "launches": n_apply,
                     "bytes_per_launch": "48 N_q + 16 N"},
        "per_degree": per_p,
    }
    fd_flops = sum((12 * max(probs[p]["n"]) * probs[p]["N"] + probs[p]["N"]) * len(rec[p]["fd_ms"]["f64"]) for p in keys)
    fd_s = sum(sum(rec[p]["fd_ms"]["f64"]) for p in keys) / 1e3
    fd_tf = fd_flops / fd_s / 1e12
    out["roofline_fd"] = {"bound": "mfma", "achieved": round(fd_tf, 3), "peak": MFMA_PEAK_TFLOPS["f64"],
                          "unit": "TFLOP/s", "frac": round(fd_tf / MFMA_PEAK_TFLOPS["f64"], 4), "dtype": "f64",
                          "kernel": "fd_xy_pass / fd_z_pass (FP64, one FD application = 3 launches)",
                          "flops_per_launch": "12 n N + N per application"}
    all_ap = np.concatenate([np.asarray(rec[p]["launch_ms"]) for p in keys])
    out["apply_ms_percentiles"] = {"of": "applies timed one launch at a time (HIP events around each)",
                                   "p10_over_mean": round(float(np.percentile(all_ap, 10) / np.mean(all_ap)), 4),
                                   "p90_over_mean": round(float(np.percentile(all_ap, 90) / np.mean(all_ap)), 4)}
    if large:
        out["large_workloads"] = large
    if react is not None:
        R = react
        Nr, Nqr = R["dp"].A.N, R["dp"].A.Nq
        t_ap, t_k = float(np.mean(R["apply_ms"])), float(np.mean(R["kernel_ms"]))
        base = per_p.get(f"p{args.reaction_degree}")
        rr = {"N": Nr, "Nq": Nqr,
              "workload": f"thick quarter ring, {args.n_el}^3 elements, p = {args.reaction_degree}, "
                          f"alpha = {10 * args.n_el ** 2} (1 + 0.5 sin(pi x1) cos(pi x2) + 0.25 x3^2), "
                          f"FD shift mean(alpha det J) = {R['sigma']:.4g}",
              "apply_ms": round(t_ap, 4), "kernel_ms": round(t_k, 4), "apply_GDOFs": round(Nr / t_ap / 1e6, 3),
              "bytes_per_launch": "56 N_q + 16 N",
              "kernel_GBs": round((56 * Nqr + 16 * Nr) / t_k / 1e6, 1),
              "kernel_frac_of_hbm_peak": round((56 * Nqr + 16 * Nr) / t_k / 1e6 / HBM_PEAK_GBS, 4),
              "kernel_traffic_bytes": committed_traffic([args.reaction_degree], reaction=True)}
        if base is not None:
            rr["kernel_time_vs_stiffness_only"] = round(t_k / base["kernel_ms"], 3)
        if not args.no_solve:
            rr.update({"fp64_solve_ms": round(float(np.median(R["fp64_ms"])), 2),
                       "fp64_iters": int(np.median(R["fp64_it"])),
                       "mixed_solve_ms": round(float(np.median(R["mix_ms"])), 2),
                       "mixed_inner": int(np.median(R["mix_inner"]))})
        out["reaction"] = rr
    if gauss:
        gd = {}
        for gp, g in gauss.items():
            alg = 48 * g["Nq"] + 16 * g["N"]
            e = {"Nq": g["Nq"], "apply_ms": round(g["apply_ms"], 4), "kernel_ms": round(g["kernel_ms"], 4),
                 "apply_GDOFs": round(g["N"] / g["apply_ms"] / 1e6, 3),
                 "kernel_GBs": round(alg / g["kernel_ms"] / 1e6, 1),
                 "kernel_frac_of_hbm_peak": round(alg / g["kernel_ms"] / 1e6 / HBM_PEAK_GBS, 4),
                 "setup_s": round(g["setup_s"], 2)}
            wq_p = per_p.get(f"p{gp}")
            if wq_p is not None:
                e["Nq_vs_wq"] = round(g["Nq"] / wq_p["Nq"], 2)
                e["apply_time_vs_wq"] = round(g["apply_ms"] / wq_p["apply_ms"], 2)
            gd[f"p{gp}"] = e
        out["gauss_quadrature"] = {
            "workload": f"thick quarter ring, {args.n_el}^3 elements, K = I, the same operator with p + 1 "
                        f"Gauss points per element (wq_setup_gauss), FP64 apply through the same fused kernels",
            "bytes_per_launch": "48 N_q + 16 N", "per_degree": gd}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(args.cpu_budget, args.cpu_solve_budget)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
