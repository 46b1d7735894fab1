"""Benchmark: time to a 1e-10 relative residual (hierarchical factorization + PCG) on the
64^3 constant-coefficient Poisson problem (n = 262,144, 7-point stencil, leaf 64,
eps = 1e-2, GC-constant, FP64), one MI355X.

A step is one whole solve with the inputs already in HBM: hsolve_factor on the CSR values,
then PCG preconditioned by the factor from x0 = 0 until ||b - A x|| <= 1e-10 ||b||. The
symbolic analysis (host, pattern only) is done once before timing and reported apart.

Prints one JSON line: the metric, per-step time, the roofline of the kernel that takes
the most time (HIP events around its launches inside the timed region), and the FP64 CPU
oracle timed on a bounded sample of the same workload family.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-1e-10 residual (factor+PCG), 64^3 Poisson; solves/s + p99 latency"

# Peaks of one MI355X (public figures): HBM3E 8 TB/s; FP64 on the vector ALUs and on the
# matrix cores both 78.6 TFLOP/s.
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6

KERNEL_BOUND = {        # kernel -> (bound, unit of its work counter)
    "k_gemm": ("alu", "flop"),
    "k_chol_inv": ("alu", "flop"),
    "k_chol_inv_blk": ("alu", "flop"),
    "k_comp_reduce<true, 128>": ("alu", "flop"),
    "k_comp_reduce<false, 512>": ("alu", "flop"),
    "k_fwd": ("hbm", "byte"),
    "k_bwd": ("hbm", "byte"),
    "k_spmv": ("hbm", "byte"),
    "k_copy": ("hbm", "byte"),
}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "c3_poisson3d_64_fp64_hbm_traffic.txt")


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE runs, scaled by a copy of known size); None when the summary is missing or the
    library sources have changed since the counters were taken."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    from paper_1611_03189_amd.profile_summary import source_hashes
    if d.get("sources") != source_hashes():
        return None
    v = d.get("kernels", {}).get(kernel)
    return None if v is None else round(float(v["hbm_bytes"]), 1)


def _oracle_solve(N: int) -> tuple[float, float, int, float, int]:
    """The FP64 oracle's factor + PCG on N^3 Poisson (leaf 64, eps 1e-2, GC), one BLAS thread;
    returns factor seconds, PCG seconds, iterations, true relative residual, n."""
    import numpy as np  # noqa: F401
    import oracle as O
    from paper_1611_03189_amd import problems as pb
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:                                  # pragma: no cover
        threadpool_limits = None
    import contextlib
    p = pb.poisson(N, 3)
    A = p.to_scipy()
    b = pb.rhs(p.n, 1, 2003)[:, 0]
    ctx = threadpool_limits(1) if threadpool_limits else contextlib.nullcontext()
    with ctx:
        t0 = time.perf_counter()
        F = O.factor(p.row_ptr, p.col_idx, p.values, p.coords, leaf=64, eps=1e-2, variant=O.GC)
        t1 = time.perf_counter()
        print(f"cpu baseline: {N}^3 oracle factor {t1 - t0:.1f} s", file=sys.stderr, flush=True)
        x, its, rel = O.pcg(A, b, lambda r: O.apply(F, r), tol=1e-10)
        t2 = time.perf_counter()
    return t1 - t0, t2 - t1, its, rel, p.n


def cpu_baseline(H, pb, torch, flops_64: float, full: bool = False) -> dict:
    """The FP64 CPU oracle on the host cores of this machine, one BLAS thread (the mode the oracle
    is written for: its dense blocks are small, and eight BLAS threads measured 2.7x slower on
    48^3). Default: a bounded sample, the whole solve of 40^3 Poisson (n = 64,000, same leaf,
    eps, GC and PCG tolerance), scaled to 64^3 by the ratio of the factorization flops the
    library counts for the two sizes (the oracle runs the same dense operations). With full,
    the 64^3 oracle solve itself is timed (about two minutes)."""
    N = 64 if full else 40
    tf, tp, its, rel, n = _oracle_solve(N)
    if full:
        scale, ratio_txt = 1.0, "no scaling"
    else:
        p = pb.poisson(N, 3)
        S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=64, eps=1e-2, variant="gc")
        S.factor(torch.from_numpy(p.values).cuda())
        flops_n = S.stats()["factor_flops"]
        S.close()
        scale = flops_64 / flops_n
        ratio_txt = f"x{scale:.2f} = counted factorization flops of 64^3 / {N}^3 ({flops_64:.3e} / {flops_n:.3e})"
    return {
        "value": round((tf + tp) * scale * 1e3, 1),
        "unit": "ms",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{N}^3 Poisson (n={n}), leaf 64, eps 1e-2, GC, FP64 oracle: factor {tf:.2f} s + PCG {tp:.2f} s "
                   f"({its} its, true rel {rel:.1e}), one BLAS thread; {ratio_txt}; host os.cpu_count() = "
                   f"{os.cpu_count()}"),
    }


def serving(count: int, slots: int, mixed: bool = True) -> dict:
    """The serving stream (mixed 2-D / 3-D lognormal systems, 1..8 right-hand sides each):
    first closed loop (every request waiting at t = 0, saturation), then open loop with
    Poisson arrivals at 0.7 x the closed-loop request rate. Latency runs from arrival to the
    last right-hand side solved; the systems are generated before the timed runs. With the
    mixed form, the same requests also run closed loop in plain FP64 (FP64 factorization and
    PCG), for the comparison on the same matrices."""
    from paper_1611_03189_amd import problems as pb
    from paper_1611_03189_amd.serve import RequestLoop, requests_from_stream
    specs = pb.serving_stream(count, seed=4)
    reqs = requests_from_stream(specs)
    loop = RequestLoop(slots=slots, mixed=mixed)
    loop.run(reqs[:min(4, len(reqs))], realtime=False)          # warm-up
    closed = loop.run(reqs, realtime=False).stats()
    rate = 0.7 * closed["requests_per_s"]
    arrivals = pb.serving_stream(count, seed=4, rate=rate)
    for r, sp in zip(reqs, arrivals):
        r.arrival = sp["arrival"]
    opened = loop.run(reqs, realtime=True).stats()
    opened["arrival_rate_per_s"] = round(rate, 3)
    out = {"workload": f"{count} systems: 2-D N~U{{64..256}} / 3-D N~U{{16..48}}, lognormal sigma 1, "
                       f"1-8 rhs, GC eps 1e-2, " + ("FP32 factorization + FP64 flexible PCG" if mixed
                                                    else "FP64 factorization + PCG") + " to 1e-10",
           "slots": slots, "closed_loop": closed, "open_loop": opened}
    if mixed:
        for r in reqs:
            r.arrival = 0.0
        loop64 = RequestLoop(slots=slots, mixed=False)
        loop64.run(reqs[:min(4, len(reqs))], realtime=False)
        closed64 = loop64.run(reqs, realtime=False).stats()
        out["fp64_closed_loop"] = closed64
        out["mixed_speedup_closed_loop"] = round(closed64["makespan_s"] / closed["makespan_s"], 3)
    return out


def variants(H, pb, np, torch, p, w, vals, b_host, x64) -> dict:
    """Other solver settings, each timed as one factor + solve after one warm-up: on the same
    64^3 system the FP32 solve phase with flexible PCG and FP64 GMRES; the 2-D lognormal 256^2
    system (sigma 2, leaf 16) in FP64 PCG and with the FP32 solve phase."""
    A3 = p.to_scipy()
    b3 = torch.from_numpy(b_host).cuda()

    def run(prob, wl, values, A, bh, bd, xref=None, **kw):
        S = H.HSolver(prob.row_ptr, prob.col_idx, coords=prob.coords, leaf=wl["leaf"], eps=wl["eps"],
                      variant="gc", tol=1e-10, **kw)
        S.factor(values)
        S.solve(bd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.factor(values)
        x, st = S.solve(bd)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        xh = x.cpu().numpy()
        r = {"ms": round(ms, 3), "factor_ms": round(st["t_factor"] * 1e3, 3),
             "solve_ms": round(st["t_solve"] * 1e3, 3), "iterations": st["iterations"],
             "true_rel_residual": float(np.linalg.norm(bh - A @ xh) / np.linalg.norm(bh)),
             "converged": st["converged"]}
        if xref is not None:
            r["rel_diff_vs_fp64_pcg"] = float(np.linalg.norm(xh - xref) / np.linalg.norm(xref))
        S.close()
        return r, xh

    out = {}
    # the mixed form: FP32 factorization (blocks, pivots, GEMMs on the FP32 matrix cores) inside
    # FP64 flexible PCG, against the FP64 PCG solution of the same system
    out["c3_fp32_factor_fpcg"], _ = run(p, w, vals, A3, b_host, b3, x64, factor_prec=32, krylov="fpcg")
    out["c3_fp32_solve_fpcg"], _ = run(p, w, vals, A3, b_host, b3, x64, apply_prec=32, krylov="fpcg")
    out["c3_gmres"], _ = run(p, w, vals, A3, b_host, b3, x64, krylov="gmres")
    p2, w2 = pb.workload("c2_lognormal2d_256")
    v2 = torch.from_numpy(p2.values).cuda()
    b2h = pb.rhs(p2.n, 1, 2002)[:, 0]
    b2 = torch.from_numpy(b2h).cuda()
    A2 = p2.to_scipy()
    out["c2_lognormal2d_256_fp64_pcg"], x2 = run(p2, w2, v2, A2, b2h, b2)
    out["c2_lognormal2d_256_fp32_solve_fpcg"], _ = run(p2, w2, v2, A2, b2h, b2, x2, apply_prec=32,
                                                       krylov="fpcg")
    out["c2_lognormal2d_256_fp32_factor_fpcg"], _ = run(p2, w2, v2, A2, b2h, b2, x2, factor_prec=32,
                                                        krylov="fpcg")
    return out


def aniso_c5(H, pb, np, torch, eps: float = 3e-3) -> dict:
    """C5, 128^3 anisotropic lognormal (sigma 3, axis factors 1, 1e-2, 1e-4; n = 2,097,152),
    leaf 64, GC, FP64 PCG to 1e-10, one factor + solve after a warm-up. The analysis bound
    (every rank at its largest, 327 GB) exceeds the device's 288 GiB, so the arena is what
    the device has free less 8 GiB; the factorization reports an error if its data would not
    fit (it uses about 246 GB)."""
    p, w = pb.workload("c5_aniso3d_128")
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=w["leaf"], eps=eps, variant="gc", tol=1e-10)
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    size = min(S.arena_bound, free - (8 << 30)) // 256 * 256
    arena = torch.empty(size, dtype=torch.uint8, device="cuda")
    v = torch.from_numpy(p.values).cuda()
    bh = pb.rhs(p.n, 1, 2003)[:, 0]
    b = torch.from_numpy(bh).cuda()
    out = {"workload": f"c5_aniso3d_128 (n={p.n}), leaf {w['leaf']}, eps {eps}, GC, FP64 PCG to 1e-10",
           "arena_bound_bytes": S.arena_bound, "arena_bytes": size}
    try:
        S.factor(v, arena=arena)
        S.solve(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.factor(v, arena=arena)
        x, st = S.solve(b)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        rel = float(np.linalg.norm(bh - p.to_scipy() @ x.cpu().numpy()) / np.linalg.norm(bh))
        out.update({"ms": round(ms, 3), "factor_ms": round(st["t_factor"] * 1e3, 3),
                    "iterations": st["iterations"], "true_rel_residual": rel, "converged": st["converged"],
                    "max_rank": S.stats()["max_rank"], "arena_used_bytes": S.stats()["device_bytes"],
                    "colours": S.stats()["colours"]})
    except H.HSolveError as e:
        out["error"] = str(e)
    S.close()
    del arena, v, b
    torch.cuda.empty_cache()
    return out


def paper_tables(H, pb, np, torch) -> dict:
    """The iteration counts of the paper's experiments (§7, Tables 1-5) on the GPU, with its
    settings: leaf red nodes of 8, the geometric well-separation rule, FD Poisson problems.
    Table 1: stationary iteration (the library stops on the true relative residual 1e-6; the
    paper stops on the relative error 1e-6). Table 2: GMRES to 1e-10, eps 0.1 (0.2, 0.3 on the
    largest grid). Table 3: 3-D GMRES, eps 0.2 / 0.3. Tables 4-5: 1e-5 inclusion and
    U(0,1] coefficients, eps 0.1 / 0.2 / 0.3 (on 512^2 instead of the paper's 1024^2).
    Columns: LoRaSp, GC-constant, GC with the smallest eigenvector (constant problems)."""
    def its(prob, eps, variant, krylov, tol=1e-10, phi=None):
        S = H.HSolver(prob.row_ptr, prob.col_idx, coords=prob.coords, leaf=8, eps=eps, variant=variant,
                      phi=phi, tol=tol, krylov=krylov, neighbours="geometric", max_iter=2000)
        try:
            S.factor(torch.from_numpy(prob.values).cuda())
            b = torch.from_numpy(pb.rhs(prob.n, 1, 7)[:, 0]).cuda()
            _, st = S.solve(b)
            return st["iterations"] if st["converged"] else f">{st['iterations']}"
        except H.NotSPD:
            return "not SPD"
        finally:
            S.close()

    out = {"settings": "leaf 8, geometric well-separation rule, GMRES tol 1e-10 (stationary: residual 1e-6)"}
    sizes = [32, 64, 128, 256, 512]
    t1, t2 = {}, {}
    for N in sizes:
        p = pb.poisson(N, 2)
        ev = pb.poisson_smallest_eigenvector(N, 2)
        t1[f"{N}^2"] = [its(p, 0.1, "lorasp", "stationary", 1e-6), its(p, 0.1, "gc", "stationary", 1e-6),
                        its(p, 0.1, "gc", "stationary", 1e-6, ev)]
        t2[f"{N}^2"] = [its(p, 0.1, "lorasp", "gmres"), its(p, 0.1, "gc", "gmres"), its(p, 0.1, "gc", "gmres", phi=ev)]
    p = pb.poisson(sizes[-1], 2)
    for e in (0.2, 0.3):
        t2[f"{sizes[-1]}^2 eps {e}"] = [its(p, e, "lorasp", "gmres"), its(p, e, "gc", "gmres")]
    out["table1_stationary_2d_eps0.1 [lorasp, gc_const, gc_eig]"] = t1
    out["table2_gmres_2d [lorasp, gc_const, gc_eig]"] = t2
    t3 = {}
    for N in (8, 16, 32):
        p = pb.poisson(N, 3)
        t3[f"{N}^3"] = [its(p, 0.2, "lorasp", "gmres"), its(p, 0.3, "lorasp", "gmres"),
                        its(p, 0.2, "gc", "gmres"), its(p, 0.3, "gc", "gmres")]
    out["table3_gmres_3d [lorasp 0.2, lorasp 0.3, gc 0.2, gc 0.3]"] = t3
    for key, prob in (("table4_inclusion_512^2", pb.piecewise_inclusion(512)),
                      ("table5_uniform_512^2", pb.uniform_random(512, 2, 1005))):
        out[key + " [lorasp, gc_const] per eps"] = {str(e): [its(prob, e, "lorasp", "gmres"), its(prob, e, "gc", "gmres")]
                                                   for e in (0.1, 0.2, 0.3)}
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-full", action="store_true",
                    help="time the oracle on 64^3 itself (about two minutes) instead of the 40^3 sample")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the other solver settings (FP32 solve phase, GMRES, 2-D lognormal 256^2)")
    ap.add_argument("--serve-requests", type=int, default=512,
                    help="requests of the serving stream (0: skip the serving measurement)")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--no-paper-tables", action="store_true",
                    help="skip the iteration counts of the paper's experiment settings")
    ap.add_argument("--c5", action="store_true",
                    help="also run C5 (128^3 anisotropic lognormal) at eps 3e-3, with an arena of what "
                         "the device has free (its analysis bound exceeds HBM)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one elementwise copy of 256 MiB first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "subtree sharding is a design note, not built.", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_1611_03189_amd import hsolve as H
    from paper_1611_03189_amd import problems as pb

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        # reads 256 MiB and writes 256 MiB: the reference for the memory counters
        xs_ = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
        ys_ = torch.empty_like(xs_)
        torch.mul(xs_, 1.0, out=ys_)
        torch.cuda.synchronize()
        del xs_, ys_
    # tile shapes of the grouped GEMM, chosen per size bucket before anything is timed
    autotune = H.tune_gemm()
    p, w = pb.workload("c3_poisson3d_64")
    b_host = pb.rhs(p.n, 1, 2003)[:, 0]
    t0 = time.perf_counter()
    S = H.HSolver(p.row_ptr, p.col_idx, coords=p.coords, leaf=w["leaf"], eps=w["eps"],
                  variant="gc", tol=1e-10)
    t_analyze = time.perf_counter() - t0
    vals = torch.from_numpy(p.values).cuda()
    b = torch.from_numpy(b_host).cuda()
    torch.cuda.synchronize()

    def step():
        S.factor(vals)
        return S.solve(b)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # one more untimed step with every kernel timed: the kernel table and the dominant kernel;
    # the timed steps then record that kernel alone (events around the others cost time)
    S.profile_begin()
    step()
    torch.cuda.synchronize()
    prof_all = S.profile_end()
    dom_name = max(prof_all, key=lambda e: e["ms"])["name"]
    S.profile_begin(only=dom_name)
    times, fac = [], []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        x, st = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        fac.append(st["t_factor"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = S.profile_end()
    ms_per_step = elapsed / args.steps * 1e3

    # the same workload with 32 right-hand sides in one batched solve (reported beside)
    B32 = torch.from_numpy(np.ascontiguousarray(pb.rhs(p.n, 32, 2103))).cuda()
    S.factor(vals)
    S.solve(B32)
    torch.cuda.synchronize()
    t32 = time.perf_counter()
    S.factor(vals)
    X32, st32 = S.solve(B32)
    torch.cuda.synchronize()
    ms32 = (time.perf_counter() - t32) * 1e3

    xs = x.cpu().numpy()
    A = p.to_scipy()
    true_rel = float(np.linalg.norm(b_host - A @ xs) / np.linalg.norm(b_host))
    stats = S.stats()

    dom = next(e for e in prof if e["name"] == dom_name)
    bound, unit = KERNEL_BOUND.get(dom["name"], ("alu", "flop"))
    per_launch_work = dom["work"] / dom["launches"]
    avg_s = dom["ms"] / dom["launches"] / 1e3
    if unit == "byte":
        achieved, peak, u = per_launch_work / avg_s / 1e9, PEAK_HBM_GBS, "GB/s"
    else:
        achieved, peak, u = per_launch_work / avg_s / 1e12, PEAK_FP64_TFLOPS, "TFLOP/s"
    roofline = {"bound": bound, "kernel": dom["name"], "achieved": round(achieved, 3),
                "peak": peak, "unit": u, "frac": round(achieved / peak, 5),
                "traffic": measured_traffic(dom["name"]), "avg_launch_ms": round(avg_s * 1e3, 4),
                "work_per_launch": round(per_launch_work, 1)}

    out = {
        "metric": METRIC,
        "value": round(ms_per_step, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "poisson3d_64^3_7pt_leaf64_eps1e-2_gc_fp64_pcg1e-10",
                   "n": p.n, "nnz": p.nnz, "leaf": w["leaf"], "eps": w["eps"], "nrhs": 1},
        "solves_per_s": round(1e3 / ms_per_step, 3),
        "step_ms": [round(t * 1e3, 3) for t in times],
        "factor_ms": round(float(np.median(fac)) * 1e3, 3),
        "pcg_iterations": stats["iterations"],
        "true_rel_residual": true_rel,
        "analyze_s": round(t_analyze, 3),
        "factor_gflop": round(stats["factor_flops"] / 1e9, 2),
        "factor_bytes": stats["factor_bytes"],
        "apply_bytes": stats["apply_bytes"],
        "max_rank": stats["max_rank"],
        "nrhs32": {"ms": round(ms32, 3), "ms_per_rhs": round(ms32 / 32, 3),
                   "pcg_iterations_max": st32["iterations"], "converged": st32["converged"]},
        "roofline": roofline,
        "autotune": {"gemm_choice_per_bucket": autotune["choice"], "shapes": autotune["shapes"]},
        "arena_bound_bytes": S.arena_bound,
        "arena_used_bytes": stats["device_bytes"],
        "kernels_untimed_step": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in e.items()}
                                 for e in sorted(prof_all, key=lambda e: -e["ms"])],
    }
    if not args.no_variants:
        out["variants"] = variants(H, pb, np, torch, p, w, vals, b_host, xs)
    if not args.no_paper_tables:
        out["paper_tables"] = paper_tables(H, pb, np, torch)
    if args.serve_requests > 0:
        out["serving"] = serving(args.serve_requests, args.serve_slots)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(H, pb, torch, stats["factor_flops"], full=args.cpu_baseline_full)
    S.close()
    if args.c5:
        out["c5"] = aniso_c5(H, pb, np, torch)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
