"""Benchmark of the numeric triple product C = P^T A P on one MI355X.

Workload (timed step): the geometric multigrid level of a 128^3 27-point operator with
lognormal(0,1) cell coefficients (seed 1) and trilinear interpolation to 64^3, in FP64 CSR.
One step is one numeric all-at-once product (merged form, K = 1, owner fold): every value of
C is computed from the values of A and P, with the symbolic phase done once beforehand, as the
paper runs one symbolic and many numerics (Section 4.1).  All inputs are resident in HBM
before the timed region.

value = algorithmic bytes of one numeric product / time per step, where the algorithmic bytes
read A and P once (int32 column + FP64 value + int32 row pointer) and write C's values once:
    B = 12 nnz(A) + 4 (n+1) + 12 nnz(P) + 4 (n+1) + 8 nnz(C).

Printed beside it (one JSON line): the roofline of the dominant kernel, the CPU oracle on the
host, the symbolic time, the two-step method, the all-at-once / merged forms with K = 8
virtual blocks, the atomic fold, peak extra device memory of each algorithm, and forward +
backward time of the differentiable form on a 64^3 problem.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def algorithmic_bytes(n, nnzA, nnzP, nnzC):
    return 12 * nnzA + 4 * (n + 1) + 12 * nnzP + 4 * (n + 1) + 8 * nnzC


PROFILE = os.path.join(ROOT, "profiles", "owner_numeric_128cubed_27pt.md")
# the kernel, and the host code and symbolic kernels that decide its tiles and their row order
KERNEL_SOURCES = ["paper_1905_08423_amd/csrc/owner.hip", "paper_1905_08423_amd/csrc/short_rows.hpp",
                  "paper_1905_08423_amd/csrc/device.hpp", "paper_1905_08423_amd/csrc/internal.hpp",
                  "paper_1905_08423_amd/csrc/kernels.hip", "paper_1905_08423_amd/csrc/api.cpp",
                  "paper_1905_08423_amd/csrc/host_logic.hpp", "paper_1905_08423_amd/csrc/symbolic.hip"]


def profiled_traffic():
    """HBM bytes per launch of the owner kernel from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), or None when the kernel's
    sources have changed since the counters were taken."""
    import hashlib

    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines()
                  if line.startswith(("traffic_bytes_per_launch:", "kernel_source_sha256:")))
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if fields.get("kernel_source_sha256", "").strip() != h.hexdigest():
        return None
    return int(float(fields["traffic_bytes_per_launch"]))


# Single-kernel runs for counter profiles: (workload, plan options, block size, adjoint)
PROFILE_CASES = {
    "c2_owner": ("c2", dict(algo="merged", fold="owner"), 1, False),
    "c2_atomic": ("c2", dict(algo="merged", fold="atomic"), 1, False),
    "c2_twostep": ("c2", dict(algo="twostep"), 1, False),
    "c3b_owner": ("c3b", dict(algo="merged", fold="owner"), 1, False),
    "c3b_atomic": ("c3b", dict(algo="merged", fold="atomic"), 1, False),
    "c3b_twostep": ("c3b", dict(algo="twostep"), 1, False),
    "c3c_bsr": ("c3c", dict(), 4, False),
    "c3c_scalar_owner": ("c3c", dict(algo="merged", fold="owner"), 1, False),
    "c5_adjoint": ("c5", dict(algo="merged", backward=True), 1, True),
}


def profile_case(lib, gen, torch, dev, name, steps, warmup):
    wl, opts, bs, adjoint = PROFILE_CASES[name]
    A, P, _ = gen.galerkin_workload(wl)
    if bs > 1:
        A, P = gen.csr_to_bsr(A, bs), gen.csr_to_bsr(P, bs)
        n, m, Aval, Pval = A.nb, P.mb, A.val.reshape(-1), P.val.reshape(-1)
    else:
        n, m, Aval, Pval = A.n_rows, P.n_cols, A.val, P.val
    d = lambda a, t: torch.as_tensor(np.ascontiguousarray(a), dtype=t).to(dev)  # noqa: E731
    plan = lib.Plan(n, m, d(A.rowptr, torch.int32), d(A.col, torch.int32), d(P.rowptr, torch.int32),
                    d(P.col, torch.int32), block_size=bs, **opts)
    Av, Pv = d(Aval, torch.float64), d(Pval, torch.float64)
    C = plan.numeric(Av, Pv)
    dC = torch.ones_like(C) if adjoint else None
    step = (lambda: plan.backward(Av, Pv, dC)) if adjoint else (lambda: plan.numeric(Av, Pv, C))
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    st = plan.stats()
    print(json.dumps({"profile_case": name, "ms_per_step": round(e0.elapsed_time(e1) / steps, 4),
                      "fold_used": st["fold_used"], "n_tiles": st["n_tiles"], "rows_formed": st["rows_formed"],
                      "nnz_C": st["nnz_C"]}), flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--side", type=int, default=128, help="fine grid side of the timed workload")
    ap.add_argument("--headline-only", action="store_true",
                    help="time only the headline numeric (for profiler runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fwd-bwd-only", action="store_true",
                    help="time only the differentiable form (forward + adjoint, for profiler runs)")
    ap.add_argument("--twostep-only", action="store_true",
                    help="time only the two-step numeric on the workload (for profiler runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain device copy of known size (counter calibration) and exit")
    ap.add_argument("--profile-case", choices=sorted(PROFILE_CASES),
                    help="run one plan's numeric (or adjoint) --warmup + --steps times and exit: "
                         "the workloads the counter summaries under profiles/ are taken on")
    ap.add_argument("--symbolic-only", action="store_true",
                    help="build the headline plan (merged, owner fold, K = 1) --warmup + --steps times "
                         "with no numeric (for profiler runs of the symbolic phase) and exit")
    ap.add_argument("--size-sweep", type=int, nargs="+", metavar="SIDE",
                    help="time the headline form (merged, owner fold, K = 1) on the 27-point "
                         "lognormal workload at each fine grid side, one JSON line per side, and exit")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1905_08423_amd as lib
    import ptap_inputs as gen

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")

    if args.copy_calibration:
        nbytes = 1 << 30
        x = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes}))
        return

    if args.profile_case:
        profile_case(lib, gen, torch, dev, args.profile_case, args.steps, args.warmup)
        return

    if args.fwd_bwd_only:
        print(json.dumps(fwd_bwd(lib, gen, torch, dev)))
        return

    if args.size_sweep:
        for side in args.size_sweep:
            print(json.dumps(size_point(lib, gen, torch, dev, side, args.steps)), flush=True)
        return

    t0 = time.time()
    side = args.side
    A = gen.stencil27(side, seed=1)
    P = gen.trilinear(side)
    gen_s = time.time() - t0
    n, m = A.n_rows, P.n_cols
    d = lambda a, t: torch.as_tensor(np.ascontiguousarray(a), dtype=t).to(dev)  # noqa: E731
    A_rowptr, A_col, A_val = d(A.rowptr, torch.int32), d(A.col, torch.int32), d(A.val, torch.float64)
    P_rowptr, P_col, P_val = d(P.rowptr, torch.int32), d(P.col, torch.int32), d(P.val, torch.float64)
    torch.cuda.synchronize()
    print(f"# workload {side}^3 27-point -> {gen.coarse_side(side)}^3: n={n} m={m} nnzA={A.nnz} "
          f"nnzP={P.nnz} (generated in {gen_s:.1f}s)", file=sys.stderr, flush=True)

    def make_plan(**kw):
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        torch.cuda.reset_peak_memory_stats()
        ts = time.perf_counter()
        plan = lib.Plan(n, m, A_rowptr, A_col, P_rowptr, P_col, **kw)
        torch.cuda.synchronize()
        sym_ms = (time.perf_counter() - ts) * 1e3
        C = plan.numeric(A_val, P_val)
        torch.cuda.synchronize()
        peak = torch.cuda.max_memory_allocated()
        st = plan.stats()
        c_bytes = 8 * st["nnz_C"] + st["pattern_bytes"]
        extra = peak - base - c_bytes
        return plan, C, sym_ms, extra

    def time_numeric(plan, C, steps, warmup):
        stream = torch.cuda.current_stream()
        for _ in range(warmup):
            plan.numeric(A_val, P_val, C)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t_start = time.perf_counter()
        for e0, e1 in evs:
            e0.record(stream)
            plan.numeric(A_val, P_val, C)
            e1.record(stream)
        torch.cuda.synchronize()
        wall_ms = (time.perf_counter() - t_start) * 1e3 / steps
        per = [e0.elapsed_time(e1) for e0, e1 in evs]
        time_numeric.median = float(np.median(per))
        return wall_ms, float(np.mean(per)), float(np.min(per))

    if args.symbolic_only:
        times = []
        for k in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p_sym = lib.Plan(n, m, A_rowptr, A_col, P_rowptr, P_col, algo="merged", fold="owner")
            torch.cuda.synchronize()
            if k >= args.warmup:
                times.append((time.perf_counter() - t0) * 1e3)
            p_sym.close()
        print(json.dumps({"symbolic_only": True, "plans": len(times), "symbolic_ms_median": round(float(np.median(times)), 3),
                          "symbolic_ms": [round(x, 3) for x in times]}), flush=True)
        return

    if args.twostep_only:
        plan, C, sym_ms, extra = make_plan(algo="twostep")
        wall_ms, ev_ms, ev_min = time_numeric(plan, C, args.steps, args.warmup)
        print(json.dumps({"twostep_numeric_ms": round(ev_ms, 4), "symbolic_ms": round(sym_ms, 2),
                          "peak_extra_mb": round(extra / 2**20, 2)}))
        return

    # ---------------- headline: merged (K = 1) owner fold.  The process's first plan also pays
    # one-time costs (page-locked staging buffers, code object loading); it is timed and released
    # first, so symbolic_ms is the time of a plan built after it.
    torch.cuda.synchronize()
    t_first = time.perf_counter()
    lib.Plan(n, m, A_rowptr, A_col, P_rowptr, P_col, algo="merged", fold="owner").close()
    torch.cuda.synchronize()
    sym_first_ms = (time.perf_counter() - t_first) * 1e3
    # symbolic_ms: the median of three later plans (now and then one later plan of a process
    # takes about twice as long, outside the library's own stages)
    sym_samples = []
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p_extra = lib.Plan(n, m, A_rowptr, A_col, P_rowptr, P_col, algo="merged", fold="owner")
        torch.cuda.synchronize()
        sym_samples.append((time.perf_counter() - t0) * 1e3)
        p_extra.close()
    plan, C, sym_ms_headline, extra_aao = make_plan(algo="merged", fold="owner", nblocks=1)
    sym_samples.append(sym_ms_headline)
    sym_ms = sorted(sym_samples)[1]
    st = plan.stats()
    nnzC = st["nnz_C"]
    B = algorithmic_bytes(n, A.nnz, P.nnz, nnzC)
    wall_ms, ev_ms, ev_min = time_numeric(plan, C, args.steps, args.warmup)
    ev_median = time_numeric.median
    value = B / (wall_ms * 1e-3) / 1e9
    achieved = B / (ev_ms * 1e-3) / 1e9
    print(f"# headline numeric: {wall_ms:.3f} ms/step wall, {ev_ms:.3f} ms mean / {ev_min:.3f} ms min "
          f"per launch (events) -> {value:.0f} GB/s", file=sys.stderr, flush=True)

    out = {
        "metric": "PtAP numeric GB/s & % HBM roofline; fwd+bwd ms; peak extra mem vs two-step",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"galerkin_{side}^3_27pt_lognormal_seed1_trilinear_to_{gen.coarse_side(side)}^3",
                   "algo": "merged all-at-once (K=1, owner fold)", "n": n, "m": m, "nnz_A": A.nnz,
                   "nnz_P": P.nnz, "nnz_C": nnzC, "algorithmic_bytes": B},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": profiled_traffic() if side == 128 else None,
                     "kernel": "k_owner_fast (owner fold, short rows)", "launch_ms_mean": round(ev_ms, 4),
                     "launch_ms_median": round(ev_median, 4), "launch_ms_min": round(ev_min, 4),
                     "measured_read_GBps": stream_read_gbps(lib, torch, dev)},
        "symbolic_ms": round(sym_ms, 2),
        "symbolic_ms_samples": [round(x, 2) for x in sym_samples],
        "symbolic_ms_first_plan_of_process": round(sym_first_ms, 2),
        "rows_formed_per_numeric": st["rows_formed"],
        "rows_needed": st["rows_needed"],
        "fold_terms": st["fold_terms"],
        "n_tiles": st["n_tiles"],
        "peak_extra_mb": {"merged_owner": round(extra_aao / 2**20, 2)},
        "plan_peak_mb_library": {"merged_owner": round(st["peak_bytes"] / 2**20, 2)},
    }
    plan.close()
    del C

    if not args.headline_only:
        variants = [("allatonce_K8_owner", dict(algo="allatonce", fold="owner", nblocks=8)),
                    ("merged_K8_owner", dict(algo="merged", fold="owner", nblocks=8)),
                    ("allatonce_K64_owner", dict(algo="allatonce", fold="owner", nblocks=64)),
                    ("merged_K64_owner", dict(algo="merged", fold="owner", nblocks=64)),
                    ("merged_owner_cached", dict(algo="merged", fold="owner", nblocks=1, cache=True)),
                    ("merged_atomic", dict(algo="merged", fold="atomic", nblocks=1)),
                    ("twostep", dict(algo="twostep"))]
        cmp_ms, cmp_sym = {}, {}
        for name, kw in variants:
            p2, C2, s_ms, extra = make_plan(**kw)
            w_ms, e_ms, _ = time_numeric(p2, C2, max(3, args.steps // 4), 2)
            cmp_ms[name] = round(e_ms, 4)
            cmp_sym[name] = round(s_ms, 2)
            out["peak_extra_mb"][name] = round(extra / 2**20, 2)
            out["plan_peak_mb_library"][name] = round(p2.stats()["peak_bytes"] / 2**20, 2)
            if name == "allatonce_K8_owner":
                out["rows_formed_allatonce_K8"] = p2.stats()["rows_formed"]
            if name == "merged_owner_cached":
                out["cache_mb"] = round(p2.stats()["cache_bytes"] / 2**20, 2)
            print(f"# {name}: numeric {e_ms:.3f} ms, symbolic {s_ms:.1f} ms, peak extra {extra / 2**20:.1f} MB",
                  file=sys.stderr, flush=True)
            p2.close()
            del C2
            torch.cuda.empty_cache()
        out["numeric_ms"] = {"merged_owner": round(ev_ms, 4), **cmp_ms}
        out["symbolic_ms_by_algo"] = cmp_sym
        out["memory_ratio_twostep_over_allatonce"] = round(
            out["peak_extra_mb"]["twostep"] / max(out["peak_extra_mb"]["merged_owner"], 1e-9), 2)
        # the paper's protocol: one symbolic and eleven numerics, end to end
        out["one_symbolic_eleven_numerics_ms"] = {}
        for name, kw in (("merged_owner", dict(algo="merged", fold="owner")), ("twostep", dict(algo="twostep"))):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            p3 = lib.Plan(n, m, A_rowptr, A_col, P_rowptr, P_col, **kw)
            C3 = p3.numeric(A_val, P_val)
            for _ in range(10):
                p3.numeric(A_val, P_val, C3)
            torch.cuda.synchronize()
            out["one_symbolic_eleven_numerics_ms"][name] = round((time.perf_counter() - t1) * 1e3, 2)
            p3.close()
            del C3
        out["fwd_bwd_ms"] = fwd_bwd(lib, gen, torch, dev)
        out["batched"] = batched(lib, gen, torch, dev)
        out["block_4x4"] = block_workload(lib, gen, torch, dev)
        out["smoothed_aggregation_96cubed"] = sa_workloads(lib, gen, torch, dev)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, P, B)

    print(json.dumps(out), flush=True)


def stream_read_gbps(lib, torch, dev, nbytes=2 << 30, reps=10):
    """HBM read bandwidth reached by the library's plain streaming-read kernel (ptap_stream_sum)
    on a 2 GiB FP64 array: the measured counterpart of the published peak."""
    x = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    out = torch.empty(1, dtype=torch.float64, device=dev)
    for _ in range(2):
        lib.stream_sum(x, out)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        lib.stream_sum(x, out)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x
    torch.cuda.empty_cache()
    return round(nbytes / (ms * 1e-3) / 1e9, 1)


def fwd_bwd(lib, gen, torch, dev, side=64):
    """Forward numeric + backward (dA, dP) through the autograd function on a 64^3 27-point
    lognormal (seed 4) problem with trilinear interpolation to 32^3, loss sum(W o C)."""
    A = gen.stencil27(side, seed=4)
    P = gen.trilinear(side)
    d = lambda a, t: torch.as_tensor(np.ascontiguousarray(a), dtype=t).to(dev)  # noqa: E731
    plan = lib.Plan(A.n_rows, P.n_cols, d(A.rowptr, torch.int32), d(A.col, torch.int32),
                    d(P.rowptr, torch.int32), d(P.col, torch.int32), algo="merged", backward=True)
    W = d(gen.loss_weights(plan.nnz_C, seed=5), torch.float64)
    Av = d(A.val, torch.float64).requires_grad_(True)
    Pv = d(P.val, torch.float64).requires_grad_(True)

    def step():
        Av.grad = None
        Pv.grad = None
        C = lib.ptap(plan, Av, Pv)
        (C * W).sum().backward()

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    reps = 10
    t = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    total = (time.perf_counter() - t) * 1e3 / reps
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    Cf = torch.empty(plan.nnz_C, dtype=torch.float64, device=dev)
    e0.record(s)
    for _ in range(reps):
        plan.numeric(Av.detach(), Pv.detach(), Cf)
    e1.record(s)
    torch.cuda.synchronize()
    fwd = e0.elapsed_time(e1) / reps
    e0.record(s)
    for _ in range(reps):
        plan.backward(Av.detach(), Pv.detach(), W)
    e1.record(s)
    torch.cuda.synchronize()
    bwd = e0.elapsed_time(e1) / reps
    plan.close()
    return {"workload": f"{side}^3_27pt_lognormal_seed4_trilinear_to_{gen.coarse_side(side)}^3",
            "fwd_bwd_ms_autograd": round(total, 4), "fwd_ms": round(fwd, 4), "bwd_ms": round(bwd, 4)}


def _time_events(fn, reps, torch):
    s = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def size_point(lib, gen, torch, dev, side, reps):
    """The headline form at one fine grid side: numeric time by HIP events over `reps` numerics
    after 3 warm-ups, and B / t."""
    A, P = gen.stencil27(side, seed=1), gen.trilinear(side)
    d = lambda a, t: torch.as_tensor(a, dtype=t, device=dev)  # noqa: E731
    plan = lib.Plan(A.n_rows, P.n_cols, d(A.rowptr, torch.int32), d(A.col, torch.int32),
                    d(P.rowptr, torch.int32), d(P.col, torch.int32), algo="merged", fold="owner")
    Av, Pv = d(A.val, torch.float64), d(P.val, torch.float64)
    C = plan.numeric(Av, Pv)
    for _ in range(2):
        plan.numeric(Av, Pv, C)
    ms = _time_events(lambda: plan.numeric(Av, Pv, C), reps, torch)
    st = plan.stats()
    B = algorithmic_bytes(A.n_rows, A.nnz, P.nnz, st["nnz_C"])
    out = {"side": side, "n": A.n_rows, "m": P.n_cols, "nnz_A": A.nnz, "nnz_P": P.nnz,
           "nnz_C": st["nnz_C"], "numeric_ms": round(ms, 4), "GBps": round(B / ms / 1e6, 1),
           "rows_formed_per_n": round(st["rows_formed"] / A.n_rows, 3), "n_tiles": st["n_tiles"]}
    plan.close()
    del C, Av, Pv
    torch.cuda.empty_cache()
    return out


def sa_workloads(lib, gen, torch, dev):
    """96^3 anisotropic 27-point operator (eps 0.01 in z, lognormal seed 2) with smoothed
    aggregation (3x3x3 aggregates; one and two damped-Jacobi steps): merged all-at-once against
    two-step, numeric time, GB/s over the algorithmic bytes and peak extra memory."""
    d = lambda a, t: torch.as_tensor(np.ascontiguousarray(a), dtype=t).to(dev)  # noqa: E731
    res = {}
    for name, label in (("c3a", "one_jacobi_step"), ("c3b", "two_jacobi_steps")):
        A, P, _ = gen.galerkin_workload(name)
        r = {"n": A.n_rows, "m": P.n_cols, "nnz_A": A.nnz, "nnz_P": P.nnz}
        Av, Pv = d(A.val, torch.float64), d(P.val, torch.float64)
        pats = [d(A.rowptr, torch.int32), d(A.col, torch.int32), d(P.rowptr, torch.int32), d(P.col, torch.int32)]
        for algo in ("merged", "twostep"):
            torch.cuda.synchronize()
            base = torch.cuda.memory_allocated()
            torch.cuda.reset_peak_memory_stats()
            plan = lib.Plan(A.n_rows, P.n_cols, *pats, algo=algo)
            C = plan.numeric(Av, Pv)
            torch.cuda.synchronize()
            st = plan.stats()
            extra = torch.cuda.max_memory_allocated() - base - 8 * st["nnz_C"] - st["pattern_bytes"]
            for _ in range(2):
                plan.numeric(Av, Pv, C)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                plan.numeric(Av, Pv, C)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 5
            B = algorithmic_bytes(A.n_rows, A.nnz, P.nnz, st["nnz_C"])
            r["nnz_C"] = st["nnz_C"]
            r[algo + "_numeric_ms"] = round(ms, 3)
            r[algo + "_GBps"] = round(B / ms / 1e6, 1)
            r[algo + "_peak_extra_mb"] = round(extra / 2**20, 1)
            print(f"# SA {label} {algo}: numeric {ms:.3f} ms, peak extra {extra / 2**20:.1f} MB",
                  file=sys.stderr, flush=True)
            plan.close()
            del C
            torch.cuda.empty_cache()
        res[label] = r
    return res


def block_workload(lib, gen, torch, dev):
    """The 4x4-block system (96^3 nodes, anisotropic 27-point couplings, block smoothed
    aggregation): the block-sparse plan against the scalar plan on the expanded matrices."""
    A, P, _ = gen.galerkin_workload("c3c")
    Ab, Pb = gen.csr_to_bsr(A, 4), gen.csr_to_bsr(P, 4)
    d = lambda a, t: torch.as_tensor(np.ascontiguousarray(a), dtype=t).to(dev)  # noqa: E731
    res = {"workload": "96^3_nodes_4x4_blocks_27pt_aniso_lognormal_seed2_block_SA_3x3x3",
           "n_scalar": A.n_rows, "nnz_A_scalar": A.nnz, "nnz_A_blocks": Ab.nnzb, "nnz_P_blocks": Pb.nnzb}

    def run(plan, Av, Pv, reps):
        C = plan.numeric(Av, Pv)
        plan.numeric(Av, Pv, C)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.numeric(Av, Pv, C)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, plan.stats()

    for name, mk, vals, reps in (
            ("bsr", lambda: lib.Plan(Ab.nb, Pb.mb, d(Ab.rowptr, torch.int32), d(Ab.col, torch.int32),
                                     d(Pb.rowptr, torch.int32), d(Pb.col, torch.int32), block_size=4),
             (Ab.val.reshape(-1), Pb.val.reshape(-1)), 10),
            ("scalar", lambda: lib.Plan(A.n_rows, P.n_cols, d(A.rowptr, torch.int32), d(A.col, torch.int32),
                                        d(P.rowptr, torch.int32), d(P.col, torch.int32)),
             (A.val, P.val), 3)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = mk()
        torch.cuda.synchronize()
        sym = (time.perf_counter() - t0) * 1e3
        Av, Pv = d(vals[0], torch.float64), d(vals[1], torch.float64)
        ms, st = run(plan, Av, Pv, reps)
        res[name + "_numeric_ms"] = round(ms, 3)
        res[name + "_symbolic_ms"] = round(sym, 1)
        res[name + "_plan_peak_mb"] = round(st["peak_bytes"] / 2**20, 1)
        if name == "bsr":
            b2 = 16
            Bb = ((4 + 8 * b2) * Ab.nnzb + 4 * (Ab.nb + 1) + (4 + 8 * b2) * Pb.nnzb + 4 * (Pb.nb + 1)
                  + 8 * b2 * st["nnz_C"])
            res["bsr_algorithmic_bytes"] = Bb
            res["bsr_GBps"] = round(Bb / ms / 1e6, 1)
        print(f"# block 4x4 {name}: numeric {ms:.2f} ms, symbolic {sym:.0f} ms", file=sys.stderr, flush=True)
        plan.close()
        del Av, Pv
        torch.cuda.empty_cache()
    res["speedup_bsr_over_scalar"] = round(res["scalar_numeric_ms"] / res["bsr_numeric_ms"], 2)
    return res


def hierarchy_case(lib, gen, torch, dev, top, nlev):
    """Geometric hierarchy from a top^3 7-point Laplacian (trilinear P at every level, each level's
    A the previous C): the plain per-level numerics against the batch (one level after another in
    one HIP graph)."""
    d = lambda a, t: torch.as_tensor(np.ascontiguousarray(a), dtype=t).to(dev)  # noqa: E731
    sides = gen.hierarchy_sides(top, nlev)
    A0 = gen.laplacian7(sides[0])
    A_rowptr, A_col = d(A0.rowptr, torch.int32), d(A0.col, torch.int32)
    A0_val = d(A0.val, torch.float64)
    del A0
    plans, Pv, keep = [], [], []
    for s_ in sides[:-1]:
        P = gen.trilinear(s_)
        Prp, Pc = d(P.rowptr, torch.int32), d(P.col, torch.int32)
        plan = lib.Plan(P.n_rows, P.n_cols, A_rowptr, A_col, Prp, Pc, algo="merged")
        plans.append(plan)
        keep.append((A_rowptr, A_col, Prp, Pc))
        Pv.append(d(P.val, torch.float64))
        A_rowptr, A_col = plan.pattern()
    C = [torch.empty(p.nnz_C, dtype=torch.float64, device=dev) for p in plans]
    Cp = [torch.empty_like(c) for c in C]
    A_vals = [A0_val] + C[:-1]
    A_plain = [A0_val] + Cp[:-1]

    def plain_h():
        for k, p in enumerate(plans):
            p.numeric(A_plain[k], Pv[k], Cp[k])

    batch = lib.Batch(plans, levels=list(range(len(plans))))
    t_plain = _time_events(plain_h, 10, torch)
    t_batch = _time_events(lambda: batch.numeric(A_vals, Pv, C), 10, torch)
    diff = max(float(((c - cp).abs().max() / cp.abs().max().clamp_min(1e-300)).item()) for c, cp in zip(C, Cp))
    out = {"sides": [int(x) for x in sides], "products": len(plans), "plain_ms": round(t_plain, 4),
           "batched_graph_ms": round(t_batch, 4), "max_rel_diff_vs_plain": diff}
    batch.close()
    for p in plans:
        p.close()
    del C, Cp, A_vals, A_plain, keep, Pv
    torch.cuda.empty_cache()
    return out


def batched(lib, gen, torch, dev):
    """The batched form against plain per-plan launches: (i) geometric hierarchies (hierarchy_case),
    one level after another in one HIP graph; (ii) 64 independent 27-point lognormal problems
    with grid sides uniform in 12..64 (seed 3), one persistent launch."""
    d = lambda a, t: torch.as_tensor(np.ascontiguousarray(a), dtype=t).to(dev)  # noqa: E731
    res = {}
    # (i) hierarchies: 256^3 down in 6 levels (large levels), 64^3 down to 2^3 (small levels,
    # where launch overhead counts)
    for top, nlev in ((256, 6), (64, 6)):
        res[f"hierarchy_{top}cubed_{nlev}_levels"] = hierarchy_case(lib, gen, torch, dev, top, nlev)
    # (ii) independent problems; plan options tuned by measurement on the largest of them
    sides3 = gen.batch_problem_sides(64, seed=3, lo=12, hi=64)
    probs = []
    for k, (nx, ny, nz) in enumerate(sides3):
        A = gen.stencil27(int(nx), int(ny), int(nz), seed=1000 + k)
        P = gen.trilinear(int(nx), int(ny), int(nz))
        probs.append((A, P))
    big = max(range(len(probs)), key=lambda k: probs[k][0].nnz)
    A, P = probs[big]
    tp, report = lib.tune(A.n_rows, P.n_cols, d(A.rowptr, torch.int32), d(A.col, torch.int32),
                          d(P.rowptr, torch.int32), d(P.col, torch.int32), d(A.val, torch.float64),
                          d(P.val, torch.float64), candidates=lib.TUNE_CANDIDATES, base={"algo": "merged"})
    tuned = tp.tuned_options
    tp.close()
    plans, Av, Pv, keep = [], [], [], []
    for A, P in probs:
        t = (d(A.rowptr, torch.int32), d(A.col, torch.int32), d(P.rowptr, torch.int32), d(P.col, torch.int32))
        keep.append(t)
        plans.append(lib.Plan(A.n_rows, P.n_cols, *t, **tuned))
        Av.append(d(A.val, torch.float64))
        Pv.append(d(P.val, torch.float64))
    C = [torch.empty(p.nnz_C, dtype=torch.float64, device=dev) for p in plans]
    Cp = [torch.empty_like(c) for c in C]

    def plain_i():
        for k, p in enumerate(plans):
            p.numeric(Av[k], Pv[k], Cp[k])

    batch = lib.Batch(plans)
    t_plain = _time_events(plain_i, 10, torch)
    t_batch = _time_events(lambda: batch.numeric(Av, Pv, C), 10, torch)
    diff = max(float(((c - cp).abs().max() / cp.abs().max().clamp_min(1e-300)).item()) for c, cp in zip(C, Cp))
    res["independent_64_sides_12_64"] = {"products": len(plans), "fine_rows": int(sum(p.n for p in plans)),
                                         "plain_ms": round(t_plain, 4), "batched_graph_ms": round(t_batch, 4),
                                         "max_rel_diff_vs_plain": diff, "tuned_options": tuned,
                                         "tuning": report}
    batch.close()
    for p in plans:
        p.close()
    return res


def cpu_baseline(A, P, B):
    """The CPU oracle (plain C, as it stands) on the same 128^3 workload: the whole product on one
    thread, then split over the host's threads (each row of C on its own; the thread count is the
    CPUs this process may use, capped by OMP_NUM_THREADS).  `value` is the thread-parallel rate;
    the one-thread rate is reported beside it."""
    import oracle

    def timed(threads):
        t = time.perf_counter()
        r = oracle.ptap(A, P, threads=threads)
        reps = 1
        while time.perf_counter() - t < 6.0 and reps < 10:
            oracle.ptap(A, P, threads=threads)
            reps += 1
        return r, reps, (time.perf_counter() - t) / reps

    r, reps1, secs1 = timed(1)
    cores = oracle.cores()
    _, repsN, secsN = timed(cores)
    return {"value": round(B / secsN / 1e9, 4), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": f"full workload (all {P.n_cols} rows of C, {r.nnz} entries): {repsN} run(s) of "
                      f"{secsN:.3f} s on {cores} threads; one thread {B / secs1 / 1e9:.4f} GB/s "
                      f"({reps1} run(s) of {secs1:.2f} s)",
            "one_thread_GBps": round(B / secs1 / 1e9, 4), "seconds": round(secsN, 3),
            "seconds_one_thread": round(secs1, 3), "host_cpus": os.cpu_count()}


if __name__ == "__main__":
    main()
