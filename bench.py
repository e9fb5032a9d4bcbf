"""Benchmark: batched ensemble throughput of the nonlinear time-history hot path.

Workload (one GPU): 64 members on a shared 64x64x32-cube quadratic-tet mesh
(786,432 tets, 3,244,995 DOF per member), two layers with per-member lognormal
Vs and uniform gamma_ref, 12 springs per point, independent seeded incident
waves, FP64 flexible CG with the FP32 block-Jacobi PCG preconditioner, tol 1e-8.

A step is one pass of the whole hot path for all members: right-hand side,
block-Jacobi diagonal, CG solve, q and Newmark updates, multi-spring law,
receiver recording.  Inputs are resident in HBM before the timed region.

Prints one JSON line: the mixed-precision throughput (DOF-steps/s summed over
members), the same members through the plain FP64 path on the same GPU with the
relative L2 difference of their receiver velocities, the roofline of the
dominant kernel (the FP32 element-by-element operator) and the CPU oracle
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "ensemble DOF-steps/s vs plain FP64 at 1e-6 rel err; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ebe32_algorithmic_bytes(n_tets: int, n_nodes: int, members_padded: int, inner_dtype: int = 0) -> float:
    """Algorithmic bytes of one inner (FP32) operator application per
    element-member: D streamed once (bfloat16 pairs: 11 words per point, 4
    points = 176 B; FP32: 84 x 4 = 336 B; element-mean bfloat16: 11 words =
    44 B), x read once and y written once per DOF (attributed per element),
    connectivity + geometry once per element (shared by the members of a
    wavefront)."""
    d = {0: 4 * 11 * 4, 1: 4 * 21 * 4, 2: 11 * 4}[inner_dtype]
    vec = 2 * 4 * 3 * n_nodes / n_tets
    mesh = (10 * 4 + 13 * 4 + 4) / members_padded
    return d + vec + mesh


# FP32 arithmetic of one element-member of the operator (an FMA counts 2),
# counted from the kernel's source: consistent mass through corner/edge sums
# 3 x 110; strain generators E_k (20 symmetric outer products of 24) and their
# sums 522; then, with D per point, per point (x4) strain 18 + D.eps 72 +
# scaling and sum 12 + force folding onto 4 corners and 3 edges 147, and edge
# terms of the point sum 144; with one D per element, the closed form: 4 stresses
# D E_k with their sum 336, corner forces 4 x 30, edge forces 6 x 54
EBE32_FLOPS_PER_POINT_D = 3 * 110 + 522 + 4 * (18 + 72 + 12 + 147) + 144
EBE32_FLOPS_ELEMENT_D = 3 * 110 + 522 + 336 + 4 * 30 + 6 * 54
FP32_PEAK_TFLOPS = 157.3


# Algorithmic HBM bytes per DOF-step of the whole step, charging every array
# once per pass the method needs (the measurement plan of the hot path): an
# FP64 PCG iteration (operator pass with FP64 D per point, vectors) 279 B, an
# FP32 inner iteration 139 B, and per step the right-hand side 223, the
# block-Jacobi diagonal 183, the q pass 199, the Newmark update 56 and the law
# 80 N_s r + 21 r 12 + 8 (state read and written, D written in FP64 and FP32;
# r = integration points per DOF, 0.969 on the 64x64x32-cube box).
def step_bytes_per_dof(n_outer: float, n_inner: float, n_springs: int, ip_per_dof: float) -> float:
    law = 80.0 * n_springs * ip_per_dof + 21.0 * ip_per_dof * 12 + 8.0
    return 279.0 * n_outer + 139.0 * n_inner + 223.0 + 183.0 + 199.0 + 56.0 + law


def step_roofline(value: float, n_outer: float, n_inner: float, n_springs: int, ip_per_dof: float) -> dict:
    b = step_bytes_per_dof(n_outer, n_inner, n_springs, ip_per_dof)
    roof = HBM_PEAK_GBS * 1e9 / b
    return {"bound": "hbm", "bytes_per_dof_step": round(b, 1), "peak_gbs": HBM_PEAK_GBS,
            "roofline_dof_steps_per_s": roof, "frac": round(value / roof, 4),
            "iterations_per_member_step": {"outer": round(n_outer, 3), "inner": round(n_inner, 3)}}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "vec.hip"):
        with open(os.path.join(ROOT, "paper_2604_02755_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(src_hash: str, element_members_per_launch: float, cluster_blocks: int):
    """HBM bytes per launch of the inner operator's element kernel from the
    committed rocprofv3 --pmc summary (FETCH_SIZE and WRITE_SIZE scaled by
    the copy calibration), taken per element-member and applied to this run's
    launches; None if the summary was taken on other kernel sources or with
    another number of cluster blocks per CU (which changes the L2 reuse)."""
    p = os.path.join(ROOT, "profiles", "inner_operator_traffic_64x64x32.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != src_hash or d.get("cluster_blocks") != cluster_blocks:
        return None
    return round(d["element"]["bytes_per_element_member"] * element_members_per_launch, 0)


def run_gpu(mesh, prob, warmup, steps, profile, tune_steps=0, tuned=None, ctx_kw=None, fixed=None, tuning_kw=None,
            pre_steps=0, profile_steps=0):
    """Create the ensemble, step ``warmup`` and then ``pre_steps`` steps,
    autotune it over the next ``tune_steps`` steps (or apply the launch shapes
    of ``tuned`` and step as many), then time ``steps`` steps one by one
    (hipGraph replay on; per-kernel event timing only if ``profile``).
    With ``profile_steps`` > 0 a separate window of that many steps follows
    with per-kernel event timing on (which replaces graph replay by direct
    launches of the same kernels); its stats are returned as ``st["prof"]``."""
    from paper_2604_02755_amd import autotune, nlth
    import torch
    ctx = nlth.Context(0, use_torch_stream=True, **(ctx_kw or {}))
    try:
        mh = ctx.mesh(mesh)
        ens = ctx.ensemble(mh, mesh, prob)
        choice = None
        if fixed is not None:
            ens.set_tuning(fixed["ebe_block"], fixed["check_every"], 1, fixed["inner_maxit"], fixed["inner_tol"],
                           cluster_blocks=fixed.get("cluster_blocks", 0), inner_method=fixed.get("inner_method", 0),
                           tail_members=fixed.get("tail_members", -1), predictor=fixed.get("predictor", 0))
            choice = dict(fixed)
        if tuned is not None:  # the launch shapes and the initial-guess policy of the tuned mixed run
            ens.set_tuning(tuned["ebe_block"], tuned["check_every"], 1, cluster_blocks=tuned.get("cluster_blocks", 0),
                           predictor=tuned.get("predictor", 0))
        if tuning_kw:
            ens.set_tuning(**tuning_kw)
        ens.step(warmup)  # the first steps carry no wave yet: warm up before tuning
        if pre_steps > 0:  # into the regime of the timed window, so the tuning sees it too
            ens.step(pre_steps)
        if tuned is not None:
            ens.step(tune_steps)
        elif tune_steps > 0:
            done0 = ens.stats()["steps_done"]
            choice = autotune.tune(ens, mesh, prob, steps_per_trial=1, log=log)
            used = ens.stats()["steps_done"] - done0
            ens.step(max(0, tune_steps - used))
        ens.reset_stats()
        ens.set_profile(profile)
        st0 = ens.stats()
        torch.cuda.synchronize()
        step_ms = []
        t0 = time.perf_counter()
        for _ in range(steps):  # each step is synchronous; the timer reads add nothing on the device
            ts = time.perf_counter()
            ens.step(1)
            step_ms.append((time.perf_counter() - ts) * 1e3)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        st = ens.stats()
        st["step_ms"] = step_ms
        if profile_steps > 0:
            ens.reset_stats()
            ens.set_profile(True)
            ens.step(profile_steps)
            st["prof"] = ens.stats()
            ens.set_profile(False)
        out = ens.read()
        ens.close()
    finally:
        ctx.close()
    return elapsed, st0, st, out, choice


def serve_run(rate, window_s, steps_range, sizes=(32, 48, 64), max_batch=64, n_check=3, seed=4000):
    """Serving stream of single-member requests (Poisson arrivals, mixed mesh
    sizes) through the library's request loop; latency = completion - arrival.
    A few requests are re-run alone afterwards (batch invariance)."""
    from paper_2604_02755_amd import inputs as I, nlth
    reqs = I.serving_requests(rate=rate, window_s=window_s, seed=seed, sizes=sizes, steps_range=steps_range)
    meshes = {n: I.serving_mesh(n) for n in sizes}
    # the solver settings of the batched benchmark: element-mean bfloat16 D in
    # the inner operator, 12 inner CG iterations per outer iteration
    probs = [I.serving_problem(r, inner_dtype=2, inner_tol=1e-12, inner_maxit=12) for r in reqs]
    ctx = nlth.Context(0, max_batch=max_batch, use_torch_stream=False)
    lat, rcs, outs = {}, {}, {}
    try:
        mh = {n: ctx.mesh(meshes[n]) for n in sizes}
        pending = {}
        i = 0
        max_in_flight = 0
        t0 = time.perf_counter()
        last_log = t0
        while i < len(reqs) or pending:
            now = time.perf_counter() - t0
            while i < len(reqs) and reqs[i]["t"] <= now:
                tk, out = ctx.submit(mh[reqs[i]["n"]], meshes[reqs[i]["n"]], probs[i])
                pending[tk] = i
                outs[i] = out
                i += 1
            max_in_flight = max(max_in_flight, len(pending))
            for tk in list(pending):
                d, _ = ctx.poll(tk)
                if d:
                    j = pending.pop(tk)
                    lat[j] = time.perf_counter() - t0 - reqs[j]["t"]
                    rcs[j] = ctx.wait(tk, 0.0)
                    ctx.release(tk)
            if time.perf_counter() - last_log > 15:
                last_log = time.perf_counter()
                log(f"serve: t={now:.0f}s submitted {i}/{len(reqs)}, in flight {len(pending)}, done {len(lat)}")
            time.sleep(0.002)
        wall = time.perf_counter() - t0
        work = sum(meshes[r["n"]].n_dof * r["steps"] for r in reqs)
        # batch invariance: re-run a few requests alone
        inv = []
        for j in np.linspace(0, len(reqs) - 1, min(n_check, len(reqs))).astype(int):
            alone = ctx.solve_as_served(mh[reqs[j]["n"]], meshes[reqs[j]["n"]], probs[j])
            b = alone["vel"]
            inv.append(float(np.linalg.norm(outs[j]["vel"] - b) / max(np.linalg.norm(b), 1e-300)))
    finally:
        ctx.close()
    L = np.array([lat[j] for j in range(len(reqs))])
    offered = sum(meshes[r["n"]].n_dof * r["steps"] for r in reqs) / window_s
    return {"requests": len(reqs), "rate_per_s": rate, "window_s": window_s,
            "offered_dof_steps_per_s": offered, "max_in_flight": max_in_flight,
            "drain_after_last_arrival_s": wall - reqs[-1]["t"],
            "steps_range": list(steps_range), "mesh_sizes": [f"{n}x{n}x16" for n in sizes],
            "max_batch": max_batch, "p50_s": float(np.percentile(L, 50)), "p99_s": float(np.percentile(L, 99)),
            "mean_s": float(L.mean()), "failed": int(sum(1 for v in rcs.values() if v != 0)),
            "throughput_dof_steps_per_s": work / wall, "wall_s": wall,
            "batch_invariance_rel_err_max": max(inv) if inv else None}


def bench_single(args):
    """One large member (the 128x128x32-cube, three perturbed layers, 150
    springs workload): mixed and plain FP64 on the same steps, and their
    receiver-velocity difference over a longer prefix."""
    from paper_2604_02755_amd import inputs as I
    dims = tuple(int(v) for v in args.mesh.split("x")) if args.mesh != "64x64x32" else (128, 128, 32)
    pre = args.warmup
    n_total = pre + args.steps
    t0 = time.perf_counter()
    mesh, pm = I.config(1, n_steps=max(n_total, args.acc_steps), mesh_dims=dims, precision=I.PRECISION_MIXED)
    _, p64 = I.config(1, n_steps=max(n_total, args.acc_steps), mesh_dims=dims, precision=I.PRECISION_FP64)
    log(f"inputs: {mesh.n_tets} tets, {mesh.n_dof} DOF, {pm.n_springs} springs ({time.perf_counter()-t0:.1f}s)")
    res = {}
    for name, pr in (("mixed", pm), ("fp64", p64)):
        el, _, st, out, _ = run_gpu(mesh, pr, args.warmup, args.steps, not args.no_profile)
        res[name] = {"value": mesh.n_dof * args.steps / el, "ms_per_step": el / args.steps * 1e3,
                     "iters": out["iters"][0, pre:n_total].tolist(),
                     "phase_ms": {"ebe64": st["ms_ebe64"], "ebe32": st["ms_ebe32"], "gather32": st["ms_gather32"],
                                  "law": st["ms_law"], "rhs_diag_q": st["ms_other"]} if not args.no_profile else None,
                     "device_gb": st["device_bytes"] / 1e9}
        log(f"{name}: {el/args.steps*1e3:.1f} ms/step")
    acc = None
    if args.acc_steps > 0:
        vels = []
        for pr in (pm, p64):
            q = I.config(1, n_steps=args.acc_steps, mesh_dims=dims, precision=pr.precision)[1]
            vels.append(run_gpu(mesh, q, 0, args.acc_steps, False)[3]["vel"][0])
        acc = float(np.linalg.norm(vels[0] - vels[1]) / max(np.linalg.norm(vels[1]), 1e-300))
        log(f"mixed vs fp64 over {args.acc_steps} steps: {acc:.2e}")
    line = {
        "metric": METRIC, "value": res["mixed"]["value"], "unit": "DOF-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["mixed"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
        "data": "synthetic (seeded perturbed three-layer mesh and band-limited input wave)",
        "config": {"workload": f"single member: {'x'.join(map(str, dims))}-cube tet10 mesh, three perturbed "
                               f"layers, 150 springs/point, mixed FP64/FP32 CG vs plain FP64, tol 1e-8",
                   "dof": mesh.n_dof, "tets": mesh.n_tets},
        "mixed": res["mixed"], "fp64_plain": res["fp64"],
        "speedup_vs_fp64": res["mixed"]["value"] / res["fp64"]["value"],
        "mixed_vs_fp64_rel_err": acc, "acc_steps": args.acc_steps,
    }
    print(json.dumps(line), flush=True)


def bench_paged(args):
    """Ensemble whose law state does not fit the device budget: the state is
    paged through pinned host memory every step (chunk ring on two copy
    streams, overlapped with the law on other chunks)."""
    from paper_2604_02755_amd import inputs as I
    dims = tuple(int(v) for v in args.mesh.split("x"))
    n_total = args.warmup + args.steps
    mesh, prob = I.config(3, n_members=args.members, mesh_dims=dims, n_steps=n_total)
    theta_gb = mesh.n_tets * 4 * prob.n_springs * args.members * (36 + 16 * (max(prob.masing_depth, 1) - 1)) / 1e9
    log(f"paged ensemble: {args.members} members, law state {theta_gb:.1f} GB, device budget {args.hbm_budget_gb} GB")
    t0 = time.perf_counter()
    ctx_kw = dict(hbm_budget=int(args.hbm_budget_gb * 2**30), host_budget=int((theta_gb * 1.05 + 8) * 1e9),
                  paging_sets=args.paging_sets)
    el, _, st, out, _ = run_gpu(mesh, prob, args.warmup, args.steps, False, ctx_kw=ctx_kw)
    log(f"paged: {el / args.steps * 1e3:.0f} ms/step, paged={st['paged']}, member sets {st['member_sets']}, "
        f"total {time.perf_counter() - t0:.0f} s")
    value = args.members * mesh.n_dof * args.steps / el
    line = {
        "metric": METRIC, "value": value, "unit": "DOF-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
        "data": "synthetic (seeded meshes, layer properties and band-limited input waves)",
        "config": {"workload": f"paged ensemble: {args.members} members on a {args.mesh}-cube tet10 mesh, 12 "
                               f"springs/point, mixed, law state {theta_gb:.1f} GB in pinned host memory",
                   "members": args.members, "hbm_budget_gb": args.hbm_budget_gb},
        "paged": bool(st["paged"]),
        "member_sets": st["member_sets"],
        "host_link": {"h2d_gb_per_step": st["h2d_bytes"] / args.steps / 1e9,
                      "d2h_gb_per_step": st["d2h_bytes"] / args.steps / 1e9,
                      "h2d_gbps": st["h2d_bytes"] / el / 1e9, "d2h_gbps": st["d2h_bytes"] / el / 1e9},
        "device_gb": st["device_bytes"] / 1e9, "host_gb": st["host_bytes"] / 1e9,
    }
    if args.zero_copy_steps > 0 and not st["paged"]:
        log("zero-copy ablation skipped: the law state fits the device budget (not paged)")
    elif args.zero_copy_steps > 0:
        # ablation of the pipeline: the law kernel works on the pinned host
        # state over the host link (the form the footnote of Section 2.3 times)
        el_zc, _, st_zc, out_zc, _ = run_gpu(mesh, prob, args.warmup, args.zero_copy_steps, False, ctx_kw=ctx_kw,
                                             tuning_kw={"zero_copy": 1})
        ms_zc = el_zc / args.zero_copy_steps * 1e3
        k = min(args.steps, args.zero_copy_steps)
        same = bool(np.array_equal(out_zc["vel"][:, :args.warmup + k], out["vel"][:, :args.warmup + k]))
        log(f"zero-copy law: {ms_zc:.0f} ms/step, results equal to the pipelined run: {same}")
        line["zero_copy_ablation"] = {"steps": args.zero_copy_steps, "ms_per_step": ms_zc,
                                      "slowdown_vs_pipelined": ms_zc / line["ms_per_step"],
                                      "results_equal_to_pipelined": same}
    print(json.dumps(line), flush=True)


def bench_serve(args):
    """The request stream at the given rate (default: the specified 4/s over
    60 s) with records shortened by --serve-scale."""
    sc = args.serve_scale
    r = serve_run(args.serve_rate, args.serve_window, (int(500 * sc), int(2000 * sc)), max_batch=args.max_batch)
    line = {
        "metric": METRIC, "value": r["p99_s"], "unit": "s (p99 solve latency)", "n_gpus": 1, "steps": None,
        "warmup": 0, "ms_per_step": None, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32", "data": "synthetic (Poisson request stream, seeded meshes and waves)",
        "config": {"workload": f"serving: Poisson {args.serve_rate}/s over {args.serve_window} s, meshes "
                               f"{{32,48,64}}^2x16 cubes, steps x{sc} of [500, 2000], 12 springs, mixed"},
        "serving": r,
    }
    print(json.dumps(line), flush=True)


def host_cpu_info() -> dict:
    """Model, threads per core and the CPUs this process may run on."""
    model, tpc = "unknown", None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.startswith("Thread(s) per core"):
                tpc = int(ln.split(":", 1)[1])
    except Exception:
        pass
    return {"model": model, "threads_per_core": tpc, "affinity": len(os.sched_getaffinity(0))}


def calibrate(kind: str):
    """hbm: a plain copy of 1 GiB (6 dispatches), the reference for scaling
    rocprofv3's FETCH_SIZE / WRITE_SIZE counters; link: pinned host memory to
    and from the device, 2 GiB per copy, each direction alone and both at once
    on two streams (the ceiling of the law-state paging)."""
    import torch
    if kind == "hbm":
        n_bytes, reps = 1 << 30, 5
        x = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        print(json.dumps({"calibration": "hbm copy", "bytes_read": n_bytes, "bytes_written": n_bytes,
                          "dispatches": reps + 1, "gbs_read_plus_write": 2 * n_bytes / dt / 1e9}), flush=True)
        return
    n_bytes, reps = 2 << 30, 4
    h_src = torch.empty(n_bytes, dtype=torch.uint8, pin_memory=True)
    h_dst = torch.empty(n_bytes, dtype=torch.uint8, pin_memory=True)
    d_a = torch.empty(n_bytes, dtype=torch.uint8, device="cuda")
    d_b = torch.empty(n_bytes, dtype=torch.uint8, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    res = {"calibration": "pinned host link", "bytes_per_copy": n_bytes, "copies": reps}

    def timed(h2d: bool, d2h: bool) -> float:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            if h2d:
                with torch.cuda.stream(s1):
                    d_a.copy_(h_src, non_blocking=True)
            if d2h:
                with torch.cuda.stream(s2):
                    h_dst.copy_(d_b, non_blocking=True)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    timed(True, True)  # warm
    t = timed(True, False)
    res["h2d_alone_gbs"] = reps * n_bytes / t / 1e9
    t = timed(False, True)
    res["d2h_alone_gbs"] = reps * n_bytes / t / 1e9
    t = timed(True, True)
    res["both_directions_gbs_each"] = reps * n_bytes / t / 1e9
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--members", type=int, default=64)
    ap.add_argument("--mesh", type=str, default="64x64x32")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=10, help="steps of the CPU oracle sample (all host threads)")
    ap.add_argument("--cpu-single-steps", type=int, default=1, help="steps of the one-thread oracle sample")
    ap.add_argument("--acc-steps", type=int, default=150, help="--config 1: steps of the accuracy comparison")
    ap.add_argument("--accuracy-ref-tol", type=float, default=0.0,
                    help="also run plain FP64 at this CG tolerance and report both paths' error against it")
    ap.add_argument("--window-start", type=int, default=130,
                    help="steps before the timed window (warmup and autotuning included, untimed steps added): "
                         "the incident wave needs about 100 steps to fill the 32 m of soil, so the window and the "
                         "accuracy comparison cover the developed response")
    ap.add_argument("--profile-steps", type=int, default=3,
                    help="steps of the profiled window after the timed steps (per-kernel event timing)")
    ap.add_argument("--no-profile", action="store_true", help="--config 1: no per-launch event timing")
    ap.add_argument("--calibrate", choices=("hbm", "link"), default=None,
                    help="hbm: a plain device copy of known size (for the rocprofv3 counter scale); link: pinned "
                         "host <-> device copy rates, each direction alone and both at once")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (defaults)")
    ap.add_argument("--inner-dtype", type=int, default=2,
                    help="storage of the inner operator's D: 0 bfloat16 per point, 1 FP32, 2 bfloat16 element mean")
    ap.add_argument("--set-tuning", type=str, default=None,
                    help="JSON with inner_tol, inner_maxit, ebe_block, check_every: use these, no autotuner")
    ap.add_argument("--config", type=int, default=2, choices=(1, 2, 3, 4),
                    help="2: batched ensemble (default); 1: one large member; 3: paged ensemble; 4: serving")
    ap.add_argument("--hbm-budget-gb", type=float, default=0.0, help="device budget of --config 3 (0: 90%% of free)")
    ap.add_argument("--paging-sets", type=int, default=0, choices=(0, 1, 2),
                    help="--config 3: member sets of the paged ensemble (0: the library's default, two)")
    ap.add_argument("--zero-copy-steps", type=int, default=0,
                    help="--config 3: also time this many steps with the law on the host state directly (ablation)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving sub-run of --config 2")
    ap.add_argument("--serve-rate", type=float, default=4.0)
    ap.add_argument("--serve-window", type=float, default=60.0)
    ap.add_argument("--serve-scale", type=float, default=0.1, help="record-length factor of --config 4")
    ap.add_argument("--max-batch", type=int, default=64, help="serving: most members per batch")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); members shard across GPUs "
              "with no exchange, so the one-GPU rate is the per-GPU figure", file=sys.stderr)
        sys.exit(2)
    if args.calibrate:
        return calibrate(args.calibrate)
    if args.config == 1:
        return bench_single(args)
    if args.config == 3:
        return bench_paged(args)
    if args.config == 4:
        return bench_serve(args)

    from paper_2604_02755_amd import inputs as I
    dims = tuple(int(v) for v in args.mesh.split("x"))
    from paper_2604_02755_amd import autotune
    t0 = time.perf_counter()
    mesh, prob = I.config(2, n_members=args.members, mesh_dims=dims)
    prob.inner_dtype = args.inner_dtype
    fixed = json.loads(args.set_tuning) if args.set_tuning else None
    n_tune = 0 if (args.no_tune or fixed) else autotune.trial_steps(prob)
    args.pre_steps = max(0, args.window_start - n_tune - args.warmup)
    pre = n_tune + args.warmup + args.pre_steps
    n_total = pre + args.steps
    # the first samples of the 1500-step records (scaled on the full records)
    n_rec = n_total + args.profile_steps
    prob.input_acc = np.ascontiguousarray(prob.input_acc[:, :n_rec])
    prob.n_steps = n_rec
    log(f"inputs: {mesh.n_tets} tets, {mesh.n_dof} DOF/member, {args.members} members ({time.perf_counter()-t0:.1f}s)")
    ndof = mesh.n_dof
    sl = slice(pre, n_total)

    # batched mixed precision (the headline), autotuned over the first steps;
    # the timed steps replay hipGraphs with no per-kernel timing; a separate
    # profiled window of the same ensemble follows for the kernel times
    el, st0, st, out_mixed, tuned = run_gpu(mesh, prob, args.warmup, args.steps, False, n_tune, fixed=fixed,
                                            pre_steps=args.pre_steps, profile_steps=args.profile_steps)
    value = args.members * ndof * args.steps / el
    log(f"mixed: {el/args.steps*1e3:.1f} ms/step, {value:.3e} DOF-steps/s, tuning {tuned and {k: tuned.get(k) for k in ('predictor', 'inner_method', 'inner_tol', 'inner_maxit', 'ebe_block', 'check_every', 'cluster_blocks', 'tail_members')}}")
    log("mixed step ms: " + " ".join(f"{x:.0f}" for x in st["step_ms"]))
    sp = st.get("prof")
    psl = slice(n_total, n_total + args.profile_steps)
    ip_per_dof = 4.0 * mesh.n_tets / ndof
    n_out = float(out_mixed["iters"][:, sl, 0].mean())
    n_in = float(out_mixed["iters"][:, sl, 1].mean())
    step_roof = step_roofline(value, n_out, n_in, prob.n_springs, ip_per_dof)

    # roofline of the dominant kernel, the inner operator's element kernel,
    # from the profiled window (per-launch HIP events on the library's compute
    # stream; the node gather that completes each application is a separate,
    # HBM-bound kernel, reported beside it).  The bound follows from the
    # arithmetic intensity: FP32 ALU when flops per algorithmic byte exceed the
    # ridge point (157.3 TFLOP/s / 8 TB/s), HBM else.
    roofline = None
    if sp and sp["n_ebe32"] > 0 and sp["ms_ebe32"] > 0:
        inner = out_mixed["iters"][:, psl, 1].astype(np.int64).sum()
        per_unit = ebe32_algorithmic_bytes(mesh.n_tets, mesh.n_nodes, sp["members_padded"], prob.inner_dtype)
        # active element-members over all applications, less those of the
        # launches on the list of the last active members
        units = int(inner) * mesh.n_tets - int(sp["elems_tail32"])
        n_app = sp["n_ebe32"]
        ms = sp["ms_ebe32"]
        flops = EBE32_FLOPS_ELEMENT_D if prob.inner_dtype == 2 else EBE32_FLOPS_PER_POINT_D
        alu = flops / per_unit > FP32_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
        gbs = per_unit * units / (ms * 1e-3) / 1e9
        tfl = flops * units / (ms * 1e-3) / 1e12
        src = kernel_source_hash()
        cb = (tuned or {}).get("cluster_blocks", 3)
        tb = traffic_from_profile(src, units / n_app, cb)
        achieved, peak = (tfl, FP32_PEAK_TFLOPS) if alu else (gbs, HBM_PEAK_GBS)
        roofline = {"bound": "alu" if alu else "hbm", "achieved": round(achieved, 2), "peak": peak,
                    "unit": "TFLOP/s" if alu else "GB/s", "frac": round(achieved / peak, 4),
                    "traffic": tb,
                    "kernel": ("nlth::k_ebe_cluster<float, %d, 0, %d> (inner operator: element forces summed per "
                               "cluster in LDS)" % ({0: 1, 1: 0, 2: 4}[prob.inner_dtype], cb))
                              if sp["members_padded"] >= 64 else
                              "nlth::k_ebe<float, 1, 0, false, 1> (inner operator: element forces)",
                    "timing": f"HIP events around each launch on the compute stream, profiled window of "
                              f"{args.profile_steps} steps after the timed steps (steps {n_total + 1}-"
                              f"{n_total + args.profile_steps})",
                    "launches": int(n_app), "avg_launch_us": round(ms / n_app * 1e3, 2),
                    "algorithmic_bytes_per_launch": round(per_unit * units / n_app, 0),
                    "algorithmic_flops_per_launch": round(flops * units / n_app, 0),
                    "bytes_per_element_member": round(per_unit, 1),
                    "flops_per_element_member": flops,
                    "hbm_gbs_algorithmic": round(gbs, 1), "fp32_tflops": round(tfl, 2),
                    "fp32_nonpacked_peak": FP32_PEAK_TFLOPS / 2,
                    "fp32_nonpacked_frac": round(tfl / (FP32_PEAK_TFLOPS / 2), 4),
                    "gather_kernel": "nlth::k_gather<float, true, true> (node sums of the cluster rows, dot fused)",
                    "gather_avg_launch_us": round(sp["ms_gather32"] / max(1, sp["n_gather32"]) * 1e3, 2),
                    "operator_avg_us": round((sp["ms_ebe32"] + sp["ms_gather32"]) / n_app * 1e3, 2)}

    # plain FP64 on the same GPU, same members, same timed steps (graph replay
    # on, no per-kernel timing, as for the headline)
    fp64 = None
    if not args.no_fp64:
        prob64 = I.config(2, n_members=args.members, mesh_dims=dims, precision=I.PRECISION_FP64)[1]
        prob64.input_acc = np.ascontiguousarray(prob64.input_acc[:, :n_total])
        prob64.n_steps = n_total
        # the comparator is tuned on its own ensemble (initial guess, launch
        # shapes, convergence-check interval), over the steps before the same
        # timed window
        n_tune64 = 0 if (args.no_tune or fixed) else autotune.trial_steps(prob64)
        el64, _, st64, out64, tuned64 = run_gpu(mesh, prob64, args.warmup, args.steps, False, n_tune64,
                                                tuned=None if n_tune64 else (tuned or {"ebe_block": 256,
                                                                                       "check_every": 8}),
                                                pre_steps=args.pre_steps + n_tune - n_tune64)
        v64 = args.members * ndof * args.steps / el64
        it64 = float(out64["iters"][:, sl, 0].mean())
        # spread of the members' iteration counts: member iterations over the
        # members times the iterations of each step's slowest member (whole
        # chunks of check_every), the share of lanes a lockstep batch without
        # the compact convergence tail keeps busy
        it_t = out64["iters"][:, sl, 0].astype(np.int64)
        ce = (tuned64 or tuned or {}).get("check_every", 8) or 8
        lane_use = float(it_t.sum() / (args.members * (ce * np.ceil(it_t.max(axis=0) / ce)).sum()))
        fp64 = {"value": v64, "ms_per_step": el64 / args.steps * 1e3, "speedup": value / v64,
                "iters_per_member_step": it64,
                "tuning": ({k: tuned64.get(k) for k in ("predictor", "ebe_block", "check_every", "cluster_blocks")
                            if k in tuned64} if tuned64 else None),
                "iters_min_max": [int(it_t.min()), int(it_t.max())], "lockstep_lane_use": round(lane_use, 4),
                "step_roofline": step_roofline(v64, it64, 0.0, prob.n_springs, ip_per_dof),
                "step_ms": [round(x, 1) for x in st64["step_ms"]]}
        log(f"fp64: {el64/args.steps*1e3:.1f} ms/step, {v64:.3e} DOF-steps/s")
        # accuracy of the timed path (64 member slots: cluster operator, compact
        # tail, the tuned inner policy) against plain FP64: every member over
        # every step both runs made
        errs = []
        for m in range(args.members):
            a, b = out_mixed["vel"][m, :n_total], out64["vel"][m, :n_total]
            errs.append(float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)))
        fp64["rel_err_max"] = max(errs)
        fp64["rel_err_median"] = float(np.median(errs))
        fp64["rel_err_sample"] = (f"all {args.members} members of the headline run, steps 1-{n_total}, receiver "
                                  f"velocity, relative L2 per member")
        log(f"mixed vs fp64 over {n_total} steps, {args.members} members: max rel err {max(errs):.2e}")
        if args.accuracy_ref_tol > 0:
            # both paths against a plain FP64 run at a much tighter tolerance
            pref = I.config(2, n_members=args.members, mesh_dims=dims, precision=I.PRECISION_FP64,
                            cg_tol=args.accuracy_ref_tol)[1]
            pref.input_acc = np.ascontiguousarray(pref.input_acc[:, :n_total])
            pref.n_steps = n_total
            outr = run_gpu(mesh, pref, args.warmup, args.steps, False, n_tune,
                           tuned=tuned or {"ebe_block": 256, "check_every": 8}, pre_steps=args.pre_steps)[3]

            def rel(o):
                return [float(np.linalg.norm(o["vel"][m, :n_total] - outr["vel"][m, :n_total]) /
                              max(np.linalg.norm(outr["vel"][m, :n_total]), 1e-300)) for m in range(args.members)]
            em, ef = rel(out_mixed), rel(out64)
            fp64["vs_reference"] = {"reference": f"plain FP64 at CG tolerance {args.accuracy_ref_tol:g}, same steps",
                                    "mixed_max": max(em), "mixed_median": float(np.median(em)),
                                    "fp64_max": max(ef), "fp64_median": float(np.median(ef))}
            log(f"against FP64 at tol {args.accuracy_ref_tol:g}: mixed max {max(em):.2e} median "
                f"{np.median(em):.2e}; FP64 at 1e-8 max {max(ef):.2e} median {np.median(ef):.2e}")

    # CPU oracle on a bounded sample of the same workload: steps of member 0,
    # setup (CRS pattern, mass, faces) excluded, on the host cores the box
    # gives this job, and on one thread
    cpu = None
    if not args.no_cpu:
        import oracle
        oracle.build()
        info = host_cpu_info()
        cores = int(os.environ.get("OMP_NUM_THREADS", 0) or info["affinity"])
        oracle.set_threads(cores)
        r = oracle.run(mesh, prob, member=0, n_steps=args.cpu_steps)
        t_steps = r["seconds"] - r["setup_seconds"]
        cpu = {"value": ndof * args.cpu_steps / t_steps, "unit": "DOF-steps/s", "cores": cores,
               "kind": "oracle",
               "sample": f"member 0, steps 1-{args.cpu_steps} of the same record on the same mesh (FP64 CRS "
                         f"assembly + block-Jacobi PCG + law per step, tol 1e-8), {t_steps:.1f} s of steps, "
                         f"setup {r['setup_seconds']:.1f} s excluded",
               "cpu_model": info["model"], "threads_per_core": info["threads_per_core"],
               "cpus_in_affinity": info["affinity"]}
        log(f"cpu oracle: {cpu['value']:.3e} DOF-steps/s on {cores} threads ({info['model']})")
        if args.cpu_single_steps > 0:
            oracle.set_threads(1)
            r1 = oracle.run(mesh, prob, member=0, n_steps=args.cpu_single_steps)
            t1 = r1["seconds"] - r1["setup_seconds"]
            cpu["single_thread"] = {"value": ndof * args.cpu_single_steps / t1, "steps": args.cpu_single_steps,
                                    "seconds": round(t1, 2)}
            oracle.set_threads(cores)
            log(f"cpu oracle, one thread: {cpu['single_thread']['value']:.3e} DOF-steps/s")

    # latency: a request stream at a rate the GPU sustains, with records
    # shorter than the specified 500-2000 steps, long enough for p99 to be an
    # interpolated percentile and not the maximum
    serving = None
    if not args.no_serve:
        serving = serve_run(1.0, 65.0, (20, 60), max_batch=args.max_batch)
        log(f"serving: p50 {serving['p50_s']:.2f} s, p99 {serving['p99_s']:.2f} s over {serving['requests']} requests")

    line = {
        "metric": METRIC, "value": value, "unit": "DOF-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
        "data": "synthetic (seeded meshes, layer properties and band-limited input waves)",
        "config": {"workload": f"batched ensemble: {args.members} members on a {args.mesh}-cube tet10 mesh, "
                               f"12 springs/point, mixed FP64/FP32 CG, tol 1e-8",
                   "inner_d_storage": {0: "bfloat16 per point", 1: "FP32 per point",
                                       2: "bfloat16 element mean"}[args.inner_dtype],
                   "members": args.members, "dof_per_member": ndof, "tets": mesh.n_tets,
                   "parallelism": "members batched in one launch"},
        "iterations": {"outer_per_member_step": float(out_mixed["iters"][:, sl, 0].mean()),
                       "inner_per_member_step": float(out_mixed["iters"][:, sl, 1].mean())},
        "tuning": ({k: tuned.get(k, 0) for k in ("predictor", "inner_method", "inner_tol", "inner_maxit", "ebe_block",
                                                 "check_every", "cluster_blocks", "tail_members")
                    if k in tuned} if tuned else None),
        "timed_steps": f"steps {pre + 1}-{n_total} of the record",
        "step_ms": [round(x, 1) for x in st["step_ms"]],
        "phase_ms_per_step": ({k: round(sp[f] / args.profile_steps, 2) for k, f in
                               (("ebe64", "ms_ebe64"), ("ebe32", "ms_ebe32"), ("gather32", "ms_gather32"),
                                ("tail32", "ms_tail32"), ("law", "ms_law"), ("rhs_diag_q", "ms_other"))}
                              if sp else None),
        "step_roofline": step_roof,
        "fp64_plain": fp64,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serving": serving,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
