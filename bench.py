"""Walker local-energy throughput on one MI355X: LO route vs full Cholesky route.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Workload: the synthetic 400-site chain (60 occupied orbitals per spin, Cholesky
vectors to 1e-5, 512 walkers with noise 0.2), FP64 end to end.  A step of a
route is one pass over the whole walker batch, inputs resident in HBM:
    LO route   = green_theta + local_energy_lo
    full route = green_theta + local_energy_full
The thresholds swept are 1e-3 ... 1e-8.  The LO threshold of the headline
`value` is the largest whose every walker energy stays within 1 mHa of the
full route: max over walkers of |Re(E_LO - E_full)| <= 1 mHa (a single energy
evaluation, the paper's 1 mHa criterion in the dodecane study).  A second
figure, `value_mean_gate`, takes the largest threshold whose walker-mean error
stays within 1 mHa: |mean Re(E_LO - E_full)| plus twice its standard error.
Prints one JSON line (stdout); progress goes to stderr.

The LO step takes about half a millisecond, so the default warm-up (400 steps,
about 0.2 s of GPU work) is long enough for the GPU clocks to settle; with a
few warm-up steps the timed region runs some 10 % slower.
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

METRIC = "walker local energies/sec, LO vs full FP64 on 1 MI355X at <=1 mHa error"
PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 (matrix and vector)
PEAK_FP32_TFLOPS = 157.3  # MI355X dense FP32 matrix
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense BF16 matrix (no sparsity)
PEAK_HBM_GBS = 8000.0
GATE_HA = 1e-3
EPS_SWEEP = (1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8)


def log(msg):
    print("[bench %7.1fs] %s" % (time.perf_counter() - T0, msg), file=sys.stderr, flush=True)


T0 = time.perf_counter()


def kernel_work(M, n, nw, X=0, n_out=0, total_rows=0, pair_rows=0):
    """Algorithmic FP64 work per launch of each kernel of the two routes.

    {kernel: (bound, flops, bytes)}; flops count a real multiply-add as 2 and a
    complex one as 8 (a real x complex one as 4); bytes count every operand once.
    """
    c16, r8 = 16.0, 8.0
    return {
        # O = Psi^T phi: real x complex, M n^2 MACs
        "overlap_kernel": ("mfma", 4.0 * M * n * n * nw, nw * c16 * (M * n + n * n) + r8 * M * n),
        "overlap4_kernel": ("mfma", 4.0 * M * n * n * nw, nw * c16 * (M * n + n * n) + r8 * M * n),
        # Gauss-Jordan inverse: n^3 complex MACs, O in and O^-1 out
        "invert_kernel": ("alu", 8.0 * n ** 3 * nw, nw * 2 * c16 * n * n),
        # theta = phi O^-1: M n^2 complex MACs; phi in, theta out, O^-1 in
        "apply_kernel": ("mfma", 8.0 * M * n * n * nw, nw * c16 * (2 * M * n + n * n)),
        # each output row: one factor row (real) times Q_o (complex); n_out =
        # 4 sum_{i<j} K_ij + sum_i K_ii, i.e. 16 M sum_{i<j} K_ij + 4 M sum_i K_ii
        # flops per walker (a diagonal block needs Ubar^T Q_i only: QR_i = QL_i)
        "lo_pass1_kernel": ("mfma", 4.0 * M * n_out * nw, r8 * total_rows * M + c16 * nw * (M * n + n_out)),
        # pair dot products: J and X per stored pair, 2 complex MACs per rank
        "lo_pass2_kernel": ("hbm", 16.0 * pair_rows * nw, c16 * nw * n_out),
        # T = Lbar^T theta per Cholesky vector + the trace epilogue
        "energy_full_kernel": ("mfma", nw * X * (4.0 * n * n * M + 8.0 * n * n),
                               r8 * X * M * n + c16 * nw * M * n),
        "theta_transpose_kernel": ("hbm", 0.0, 2 * c16 * nw * M * n),
        # Eq. 17: Y^[ij] theta_j and Y^[ij] theta_i per pair i < j, one product for i = j
        "hr_energy_kernel": ("mfma", 4.0 * M * M * nw * (n * (n - 1) + n),
                             r8 * M * M * n * (n + 1) / 2 + c16 * nw * M * n),
    }


def measured_traffic(kernel, eps):
    """HBM bytes per launch (read + write) of `kernel` from the committed
    rocprofv3 counter table, if the table was taken at this threshold from the
    current source of the kernel; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            table = json.load(f)
        if float(table["epsilon"]) != float(eps):
            return None
        ent = table["kernels"][kernel]
        with open(os.path.join(ROOT, ent["source"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != ent["source_sha256"]:
                return None
        if len(ent["launches"]) != 1:
            return None
        return ent["launches"][0]["read_bytes"] + ent["launches"][0]["write_bytes"]
    except (OSError, KeyError, ValueError):
        return None


KERNEL_SOURCES = {
    "overlap_kernel": "green_theta.hip", "overlap4_kernel": "green_theta.hip", "invert_kernel": "green_theta.hip",
    "apply_kernel": "green_theta.hip",
    "lo_pass1_kernel": "energy_lo.hip", "lo_pass1_reg_kernel": "energy_lo.hip", "lo_pass2_kernel": "energy_lo.hip",
    "reduce_partials_kernel": "energy_full.hip", "energy_full_kernel": "energy_full.hip",
}


def _counter_rows(path):
    """(kernel base name, grid, counter, value) rows of every rocprofv3
    counter-collection CSV under `path`."""
    import csv
    import glob
    rows = []
    for fn in glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True):
        with open(fn) as f:
            for r in csv.DictReader(f):
                name = r["Kernel_Name"].split("(")[0].split("<")[0].split("::")[-1].strip()
                rows.append((name, int(r["Grid_Size"]), r["Counter_Name"], float(r["Counter_Value"])))
    return rows


def write_traffic_table(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, eps, workload, out_path):
    """HBM bytes per launch of each kernel from rocprofv3 FETCH_SIZE and
    WRITE_SIZE runs (KiB per dispatch), scaled by what the same counters read
    for a plain device copy of known size, with the sha256 of each kernel's
    source so that stale numbers are never used."""
    import hashlib
    copy_bytes = None

    def per_kernel(path, counter):
        acc = {}
        for name, grid, cname, val in _counter_rows(path):
            if cname.startswith(counter):
                acc.setdefault((name, grid), []).append(val * 1024.0)
        return {k: float(np.mean(v)) for k, v in acc.items()}, {k: len(v) for k, v in acc.items()}

    cf, _ = per_kernel(copy_fetch_dir, "FETCH_SIZE")
    cw, _ = per_kernel(copy_write_dir, "WRITE_SIZE")
    copy_key = max(cf, key=lambda k: cf[k])        # the 1 GiB copy is the largest dispatch
    copy_bytes = 1024.0 ** 3
    fetch_scale = copy_bytes / cf[copy_key]
    write_scale = copy_bytes / cw[max(cw, key=lambda k: cw[k])]
    fe, nf = per_kernel(fetch_dir, "FETCH_SIZE")
    wr, _ = per_kernel(write_dir, "WRITE_SIZE")
    table = {"workload": workload, "epsilon": eps, "fetch_scale": fetch_scale, "write_scale": write_scale,
             "kernels": {}}
    for (name, grid), v in sorted(fe.items()):
        if name not in KERNEL_SOURCES:
            continue
        src = os.path.join("paper_2202_00832_amd", "csrc", KERNEL_SOURCES[name])
        with open(os.path.join(ROOT, src), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
        ent = table["kernels"].setdefault(name, {"launches": [], "source": src, "source_sha256": sha})
        ent["launches"].append({"grid": grid, "dispatches": nf[(name, grid)], "fetch_kib": v / 1024.0,
                                "write_kib": wr.get((name, grid), 0.0) / 1024.0,
                                "read_bytes": v * fetch_scale, "write_bytes": wr.get((name, grid), 0.0) * write_scale})
    with open(out_path, "w") as f:
        json.dump(table, f, indent=1)
    return table


def roofline_of(name, work, ms_per_launch):
    bound, flops, nbytes = work[name]
    sec = ms_per_launch * 1e-3
    if bound == "hbm":
        ach = nbytes / sec / 1e9
        peak, unit = PEAK_HBM_GBS, "GB/s"
    else:
        ach = flops / sec / 1e12
        peak, unit = PEAK_FP64_TFLOPS, "TFLOP/s"
    return {"bound": bound, "achieved": round(ach, 3), "peak": peak, "unit": unit, "frac": round(ach / peak, 4),
            "kernel": name, "us_per_launch": round(ms_per_launch * 1e3, 2),
            "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": nbytes}


def time_route(torch, ctx, step, steps, warmup, marks):
    """`warmup` untimed steps, `steps` timed steps, then `steps` more with events.

    The first timed region holds nothing but the steps between two events and
    gives the throughput.  In the second one, `step(ev)` also records the
    per-call events of the dict `ev`, and the library records an event on its
    stream before each of its kernels; it gives the per-call split and the
    per-kernel durations.  Returns (total ms of region 1,
    {call: [ms per step]}, {kernel: (launches, total ms)}).
    """
    for _ in range(warmup):
        step(None)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        step(None)
    stop.record()
    torch.cuda.synchronize()
    total = start.elapsed_time(stop)

    evs = [{m: torch.cuda.Event(enable_timing=True) for m in marks} for _ in range(steps)]
    ctx.profile_enable(True)
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    kernels = ctx.profile_summary()
    ctx.profile_enable(False)
    split = {}
    for a, b in zip(marks[:-1], marks[1:]):
        split[a + "->" + b] = [e[a].elapsed_time(e[b]) for e in evs]
    return total, split, kernels


def hr_study(torch, ctx, lbar, trial_d, phi_d, info, energy, e_full_h, work, M, n, nw, steps=10):
    """The half-rotated ERI route (Eq. 17) on the same workload: pair-block
    build, time per step (green_theta + local_energy_hr, with theta
    orbital-major: the route reads theta columns of 32 walkers, contiguous in
    that layout) and agreement with the full route."""
    t = time.perf_counter()
    hr = ctx.build_hr_eri(lbar)
    build_s = time.perf_counter() - t
    theta_om = torch.empty((n, M, nw), dtype=torch.complex128, device="cuda")
    logov = torch.empty(nw, dtype=torch.complex128, device="cuda")
    ctx.green_theta(trial_d, phi_d, theta_om, logov, info, orbital_major=True)
    e_hr = ctx.local_energy_hr(hr, theta_om, info, orbital_major=True)
    torch.cuda.synchronize()
    diff = float(np.abs(e_hr.cpu().numpy() - e_full_h).max())

    def step(ev):
        if ev is not None:
            ev["a"].record()
        ctx.green_theta(trial_d, phi_d, theta_om, logov, info, orbital_major=True)
        if ev is not None:
            ev["b"].record()
        ctx.local_energy_hr(hr, theta_om, info, energy, orbital_major=True)
        if ev is not None:
            ev["c"].record()

    tot, split, kern = time_route(torch, ctx, step, steps, 2, ["a", "b", "c"])
    ms = tot / steps
    kernels = {k: roofline_of(k, work, t_ / c) for k, (c, t_) in kern.items() if k in work}
    log("HR-ERI: %.3f ms/step (local_energy_hr %.3f), pair blocks %.2f GB built in %.2f s, max |E_hr - E_full| %.2e"
        % (ms, float(np.mean(split["b->c"])), hr.bytes / 1e9, build_s, diff))
    out = {"value": round(nw / (ms * 1e-3), 1), "unit": "walker-energies/s", "ms_per_step": round(ms, 4),
           "local_energy_hr_ms": round(float(np.mean(split["b->c"])), 4), "steps": steps, "theta": "orbital-major",
           "pair_block_bytes": hr.bytes, "build_s": round(build_s, 3), "max_abs_diff_vs_full_Ha": diff,
           "roofline": kernels.get("hr_energy_kernel"), "kernels": kernels}
    hr.close()
    return out


def release_cached(torch, what):
    """Hands torch's cached device blocks back to the driver before a study
    that allocates outside torch's allocator (library workspaces, hipBLAS
    work arrays) and logs the free device memory."""
    import gc
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    log("%s: %.1f of %.1f GiB free on the device" % (what, free / 2 ** 30, total / 2 ** 30))


def event_ms(torch, fn, reps=50, warm=5):
    """Mean ms per call of fn() over reps calls between two events, after warm calls."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def few_walker_study(torch, ctx, lbar, trial_d, phi_d, factors, nw=16):
    """The paper's timing shape (Sec. 3, dodecane: the energy evaluation of 16
    walkers, LO at each threshold against the HR-ERI code): energy calls only,
    on the first 16 walkers of the workload."""
    phi = phi_d[:nw].contiguous()
    th, _, inf = ctx.green_theta(trial_d, phi, transposed=True)
    th_om, _, inf_om = ctx.green_theta(trial_d, phi, orbital_major=True)
    hr = ctx.build_hr_eri(lbar)
    hr_ms = event_ms(torch, lambda: ctx.local_energy_hr(hr, th_om, inf_om, orbital_major=True))
    out = {"walkers": nw, "local_energy_hr_ms": round(hr_ms, 4), "lo": {}}
    for eps, f in factors.items():
        lo_ms = event_ms(torch, lambda f=f: ctx.local_energy_lo(f, th, inf, transposed=True))
        out["lo"]["%g" % eps] = {"local_energy_lo_ms": round(lo_ms, 4), "speedup_vs_hr": round(hr_ms / lo_ms, 1)}
    hr.close()
    log("16 walkers: HR-ERI %.3f ms, LO %s" % (hr_ms, ", ".join("%s %.3f ms (%.0fx)" % (k, v["local_energy_lo_ms"],
                                                                                          v["speedup_vs_hr"])
                                                               for k, v in out["lo"].items())))
    return out


def _err_stats(e, ref):
    """Per-walker errors of E2 = E_J + E_K against the FP64 result."""
    d = np.abs(e.sum(axis=1) - ref.sum(axis=1))
    rel = d / np.maximum(np.abs(ref.sum(axis=1)), 1e-300)
    return {"max_abs_dE_Ha": float(d.max()), "mean_abs_dE_Ha": float(d.mean()),
            "p99_abs_dE_Ha": float(np.percentile(d, 99)), "median_abs_dE_Ha": float(np.median(d)),
            "max_rel_dE": float(rel.max()), "walkers_within_1e-5_Ha": round(float(np.mean(d <= 1e-5)), 4)}


def precision_study(torch, lofqmc, synth, steps, eps=1e-4):
    """The full route and the LO route (eps = 1e-4) with their contractions in
    FP64, FP32 and split BF16 on the 500-site chain (48 orbitals, 1024
    walkers): time per call and error of each walker's energy against the
    FP64 result of the same route and inputs.  The FP64 results equal the CPU
    reference to 1e-9 Ha per walker (the parity tests), so these errors are
    the errors against the reference to within 1e-9 Ha."""
    cfg = synth.CHAIN_PRECISION
    log("precision study: generating %s" % cfg.name)
    system = synth.make_system(cfg)
    M, n, nw, X = cfg.M, cfg.n, cfg.nw, system.n_chol
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    ctx = lofqmc.Context()
    chol_d = dev(system.chol)
    trial_d, phi_d = dev(system.trial), dev(system.walkers)
    lbar = ctx.build_half_rotated_chol(chol_d, trial_d)
    del chol_d
    theta, logov, info = ctx.green_theta(trial_d, phi_d)
    energy = torch.empty((nw, 2), dtype=torch.complex128, device="cuda")
    ref = ctx.local_energy_full(lbar, theta, info, precision=lofqmc.LO_FP64).cpu().numpy()
    fac = ctx.build_lo_factors(lbar, eps)
    finfo = fac.info()
    ref_lo = ctx.local_energy_lo(fac, theta, info, precision=lofqmc.LO_FP64).cpu().numpy()
    out = {"workload": cfg.name, "M": M, "n_occ": n, "n_chol": X, "walkers": nw,
           "error_reference": "the FP64 result of the same route (equal to the CPU reference within 1e-9 Ha)",
           "runs": {}, "lo": {"epsilon": eps, "mean_rank": float(finfo["ranks"].mean()),
                              "lo_fp64_vs_full_fp64": _err_stats(ref_lo, ref), "runs": {}}}
    names = {lofqmc.LO_FP64: "fp64", lofqmc.LO_FP32: "fp32", lofqmc.LO_BF16X3: "bf16x3"}
    for p in (lofqmc.LO_FP64, lofqmc.LO_FP32, lofqmc.LO_BF16X3):
        def step(ev, p=p):
            ctx.local_energy_full(lbar, theta, info, energy, precision=p)
        tot, _, kern = time_route(torch, ctx, step, steps, 1, ["a"])
        e = ctx.local_energy_full(lbar, theta, info, precision=p).cpu().numpy()
        dk = np.abs(e[:, 1] - ref[:, 1])
        r = {"ms_per_call": round(tot / steps, 3), "walker_energies_per_s": round(nw / (tot / steps * 1e-3), 1),
             **_err_stats(e, ref), "max_abs_dEK_Ha": float(dk.max()),
             "kernel_us": {k: round(t / c * 1e3, 1) for k, (c, t) in kern.items()}}
        # rooflines of the contraction kernels against the peak of the dtype
        # they run in, on the method's own flops (unpadded sizes, each product
        # counted once also where split BF16 runs it as three BF16 products):
        # the exchange contraction T = Lbar^T theta (real x complex, 4 M n^2 per
        # walker and vector) and the FP64 Coulomb traces (4 M n per walker and
        # vector)
        contraction = 4.0 * M * n * n * X * nw
        spec = {"energy_full_kernel": (contraction + 8.0 * n * n * X * nw, PEAK_FP64_TFLOPS, "fp64"),
                "exchange_lp_kernel": (contraction,
                                       PEAK_BF16_TFLOPS if p == lofqmc.LO_BF16X3 else PEAK_FP32_TFLOPS,
                                       "bf16" if p == lofqmc.LO_BF16X3 else "fp32"),
                "coulomb_trace_kernel": (4.0 * M * n * X * nw, PEAK_FP64_TFLOPS, "fp64")}
        r["kernels"] = {}
        for k, (flops, peak, dt) in spec.items():
            if k in kern:
                ach = flops / (kern[k][1] / kern[k][0] * 1e-3) / 1e12
                r["kernels"][k] = {"bound": "mfma", "dtype": dt, "achieved": round(ach, 3), "peak": peak,
                                   "unit": "TFLOP/s", "frac": round(ach / peak, 4),
                                   "us_per_launch": round(kern[k][1] / kern[k][0] * 1e3, 2),
                                   "algorithmic_flops_per_launch": flops}
        out["runs"][names[p]] = r
        log("precision full %s: %.3f ms/call, max |dE| %.2e Ha, mean %.2e, %.1f %% of walkers within 1e-5 Ha"
            % (names[p], r["ms_per_call"], r["max_abs_dE_Ha"], r["mean_abs_dE_Ha"],
               100 * r["walkers_within_1e-5_Ha"]))
        # LO route at eps, same precision
        def step_lo(ev, p=p):
            ctx.local_energy_lo(fac, theta, info, energy, precision=p)
        tot, _, kern = time_route(torch, ctx, step_lo, max(steps, 20), 3, ["a"])
        e = ctx.local_energy_lo(fac, theta, info, precision=p).cpu().numpy()
        r = {"ms_per_call": round(tot / max(steps, 20), 4),
             "walker_energies_per_s": round(nw / (tot / max(steps, 20) * 1e-3), 1), **_err_stats(e, ref_lo),
             "kernel_us": {k: round(t / c * 1e3, 1) for k, (c, t) in kern.items()}}
        out["lo"]["runs"][names[p]] = r
        log("precision LO %s: %.4f ms/call, max |dE| %.2e Ha, mean %.2e, %.1f %% of walkers within 1e-5 Ha"
            % (names[p], r["ms_per_call"], r["max_abs_dE_Ha"], r["mean_abs_dE_Ha"],
               100 * r["walkers_within_1e-5_Ha"]))
    fac.close()
    ctx.close()
    return out


def batch_study(torch, lofqmc, synth, evaluations=50):
    """Eight chain systems of uneven size (M uniform in [100, 600], n = M // 7,
    64-512 walkers): per evaluation, from the walkers of every system, FP64
    green_theta and FP32 full-route energies, one persistent exchange launch
    for all systems; `evaluations` evaluations captured in one HIP graph;
    against the same evaluations as green_theta + local_energy_full per
    system.  The autotuner scales each bucket's chunk by 1/4 ... 4."""
    from paper_2202_00832_amd import autotune
    cfgs = synth.batch_configs()
    log("batching: %s" % ", ".join(c.name for c in cfgs))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    ctx = lofqmc.Context()
    systems, total_w = [], 0
    for c in cfgs:
        sysm = synth.make_system(c)
        trial, phi = dev(sysm.trial), dev(sysm.walkers)
        lbar = ctx.build_half_rotated_chol(dev(sysm.chol), trial)
        theta, _, info = ctx.green_theta(trial, phi)
        systems.append({"lbar": lbar, "theta": theta, "info": info, "trial": trial, "phi": phi})
        total_w += c.nw
        del sysm
    torch.cuda.synchronize()
    tuned = autotune.tune(ctx, systems, factors=(0.25, 0.5, 2.0, 4.0), reps=2, log=log)
    b = lofqmc.Batch(ctx, systems, tuned["chunk"])
    b.capture(evaluations)
    b.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    b.replay()
    e1.record()
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1) / evaluations
    # the same work as separate calls, one per system and evaluation
    outs = [torch.empty((sd["theta"].shape[0], 2), dtype=torch.complex128, device="cuda") for sd in systems]
    ths = [torch.empty_like(sd["theta"]) for sd in systems]
    infs = [torch.empty_like(sd["info"]) for sd in systems]

    def separate():
        for sd, o, th, inf in zip(systems, outs, ths, infs):
            ctx.green_theta(sd["trial"], sd["phi"], th, None, inf)
            ctx.local_energy_full(sd["lbar"], th, inf, o, precision=lofqmc.LO_FP32)
    separate()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(evaluations):
        separate()
    e1.record()
    torch.cuda.synchronize()
    seq_ms = e0.elapsed_time(e1) / evaluations
    maxdiff = max(float((a - o).abs().max()) for a, o in zip(b.energies, outs))
    # FP32 exchange contraction of all systems per evaluation (4 M n^2 per
    # walker and Cholesky vector), over the whole evaluation's time (which also
    # holds the FP64 Coulomb sums and reductions)
    xflops = sum(4.0 * sd["lbar"].shape[1] * sd["lbar"].shape[2] ** 2 * sd["lbar"].shape[0] * sd["theta"].shape[0]
                 for sd in systems)
    # green_theta per walker: overlap 4 M n^2, inverse 8 n^3, apply 8 M n^2 (FP64)
    gflops = sum(sd["theta"].shape[0] * (12.0 * sd["lbar"].shape[1] * sd["lbar"].shape[2] ** 2
                                         + 8.0 * sd["lbar"].shape[2] ** 3) for sd in systems)
    info = b.info()
    b.close()
    ctx.close()
    out = {"systems": [c.name for c in cfgs], "walkers": total_w, "evaluations_per_graph": evaluations,
           "work_items": int(info["items"]), "chunk": [int(x) for x in info["chunk"]],
           "autotune_ms": {"default": round(tuned["default_ms"], 3), "tuned": round(tuned["ms"], 3),
                           "trials": len(tuned["trials"]), "factors": [0.25, 0.5, 2.0, 4.0],
                           "tuned_over_default": round(tuned["ms"] / tuned["default_ms"], 4)},
           "evaluation": "green_theta (FP64) + FP32 full route of every system, from the walkers",
           "green_theta_flops_per_evaluation": gflops,
           "graph_ms_per_evaluation": round(graph_ms, 3),
           "walker_energies_per_s": round(total_w / (graph_ms * 1e-3), 1),
           "separate_calls_ms_per_evaluation": round(seq_ms, 3),
           "max_abs_diff_vs_separate_calls_Ha": maxdiff,
           "roofline_whole_evaluation": {"bound": "mfma", "dtype": "fp32",
                                         "achieved": round(xflops / (graph_ms * 1e-3) / 1e12, 3),
                                         "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                                         "frac": round(xflops / (graph_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4),
                                         "algorithmic_flops_per_evaluation": xflops}}
    log("batching: graph %.3f ms/eval (%.0f walker-energies/s), separate calls %.3f ms/eval"
        % (graph_ms, out["walker_energies_per_s"], seq_ms))
    return out


def _orthonormalize(torch, a):
    """Orthonormal columns spanning those of each a[w] (Cholesky QR,
    a = Q L^H with L L^H = a^H a, Q = a L^{-H}).  Q differs from a Householder
    QR's only by column phases, which the circular walk noise does not see.
    L is inverted through torch.linalg.inv (LU) and applied by a batched
    product: hipBLAS's batched complex triangular solve failed here with an
    allocation error whatever the batch size."""
    ah = a.conj().transpose(-1, -2).contiguous()
    L = torch.linalg.cholesky(ah @ a)
    linv_h = torch.linalg.inv(L).conj().transpose(-1, -2).contiguous()
    return a @ linv_h


def residual_study(torch, lofqmc, synth, n_train=20480, n_test=2048, steps=2000, step_sigmas=(0.005, 0.02),
                   sketch=24):
    """Learned correction of the LO energy on the 800-site chain (100 orbitals
    per spin, 2048 walkers, eps = 1e-3): LO factors from the randomized SVD,
    exact energies from the full (Cholesky) route, walker pairs along random
    walks from the trial (walk steps 0.005 and 0.02), training on the GPU,
    held-out error of plain LO, of LO plus a constant offset (the training mean
    of the dropped energy), of LO plus the first-order term alone (a
    least-squares line in sum_i x_i3, fitted on the training pairs) and of the
    network's correction (the held-out pairs are whole walks), and the checked
    corrected-LO throughput."""
    from paper_2202_00832_amd import residual as RES
    cfg = synth.CHAIN_RESIDUAL
    eps = cfg.epsilons[0]
    log("residual study: generating %s" % cfg.name)
    base = synth.make_system(cfg, nw=1)
    M, n, nb = cfg.M, cfg.n, cfg.nw
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    ctx = lofqmc.Context()
    trial_d = dev(base.trial)
    chol_d = dev(base.chol)
    lbar = ctx.build_half_rotated_chol(chol_d, trial_d)
    del chol_d
    rng = np.random.default_rng(2025)
    t0 = time.perf_counter()
    omega = dev(rng.standard_normal((M, sketch)))
    f = ctx.build_lo_factors_randomized(lbar, eps, omega, power_iters=2)
    torch.cuda.synchronize()
    factor_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    ctx.residual_prepare(f, lbar, trial_d)
    prep_s = time.perf_counter() - t0
    exact = lambda th, inf: ctx.local_energy_full(lbar, th, inf)  # noqa: E731
    ranks = f.info()["ranks"]
    log("residual study: randomized LO factors %.2f s (<K> = %.3f), gradient set-up %.2f s"
        % (factor_s, ranks.mean(), prep_s))
    out = {"workload": cfg.name, "M": M, "n_occ": n, "n_chol": base.n_chol, "epsilon": eps,
           "factors": "randomized SVD, sketch %d, 2 power steps" % sketch, "factor_build_s": round(factor_s, 2),
           "gradient_setup_s": round(prep_s, 2), "mean_rank": float(ranks.mean()),
           "exact_route": "full Cholesky route (Eq. 16)", "features": "sum_j K_ij, sum_j m_ij, ||theta_i||, "
           "Re(g_i . theta_i) with g the gradient of E_HR - E_LO at the trial", "walks": {}}
    rms = lambda d: float(np.sqrt(np.mean(d ** 2)) * 1e3)  # noqa: E731
    mx = lambda d: float(np.abs(d).max() * 1e3)  # noqa: E731
    nsteps = -(-(n_train + n_test) // nb)
    for step_sigma in step_sigmas:
        # walker pairs along random walks phi <- QR(phi + s (Z1 + i Z2)) from the
        # trial (a stand-in for the propagation), one pair per walker and step
        gen = torch.Generator(device="cuda").manual_seed(2025)
        phi = trial_d.to(torch.complex128).unsqueeze(0).repeat(nb, 1, 1)
        X, EF, EL = [], [], []
        t0 = time.perf_counter()
        for _ in range(nsteps):
            z = torch.complex(torch.randn(phi.shape, dtype=torch.float64, device="cuda", generator=gen),
                              torch.randn(phi.shape, dtype=torch.float64, device="cuda", generator=gen))
            phi = _orthonormalize(torch, phi + step_sigma * z)
            theta, _, info = ctx.green_theta(trial_d, phi)
            EF.append(exact(theta, info))
            EL.append(ctx.local_energy_lo(f, theta, info))
            X.append(ctx.residual_features(f, theta))
        torch.cuda.synchronize()
        gen_s = time.perf_counter() - t0
        x, ef, el = torch.stack(X), torch.stack(EF), torch.stack(EL)   # [step][walker]...
        del X, EF, EL
        n_test_walks = -(-n_test // nsteps)
        tr, te = slice(0, nb - n_test_walks), slice(nb - n_test_walks, nb)
        flat = lambda t, part: t[:, part].reshape(-1, *t.shape[2:]).contiguous()  # noqa: E731
        xtr, xte = flat(x, tr), flat(x, te)
        model = RES.ResidualModel(ctx, RES.init_params(xtr.cpu().numpy(), ctx.residual_nparam(), seed=0))
        t0 = time.perf_counter()
        losses = model.train(xtr, flat(ef, tr), flat(el, tr), steps=steps, lr=1e-3, batch=1024)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t0
        e_full = ctx.residual_apply(flat(ef, te)).real.cpu().numpy()
        e_lo = ctx.residual_apply(flat(el, te)).real.cpu().numpy()
        e_net = model.corrected(flat(el, te), xte).real.cpu().numpy()
        t_tr = ctx.residual_target(flat(ef, tr), flat(el, tr)).cpu().numpy() / 1e3
        offset = t_tr.mean()
        # the first-order term alone: a least-squares line in sum_i x_i3
        s_tr = xtr[:, :, 3].double().sum(dim=1).cpu().numpy()
        s_te = xte[:, :, 3].double().sum(dim=1).cpu().numpy()
        A = np.stack([np.ones_like(s_tr), s_tr], axis=1)
        coef = np.linalg.lstsq(A, t_tr, rcond=None)[0]
        lin = coef[0] + coef[1] * s_te
        d_plain, d_const, d_lin, d_net = e_full - e_lo, e_full - e_lo - offset, e_full - e_lo - lin, e_full - e_net
        rec = {"step_sigma": step_sigma, "walk_steps": nsteps, "train_pairs": int(xtr.shape[0]),
               "test_pairs": int(xte.shape[0]), "test_walks": n_test_walks, "pair_generation_s": round(gen_s, 2),
               "train_steps": steps, "train_s": round(train_s, 2),
               "loss_first_last_standardised": [float(losses[0]), float(np.mean(losses[-50:]))],
               "heldout_rms_mHa": {"plain_lo": rms(d_plain), "constant_offset": rms(d_const),
                                   "first_order_line": rms(d_lin), "network": rms(d_net)},
               "heldout_max_abs_mHa": {"plain_lo": mx(d_plain), "constant_offset": mx(d_const),
                                       "first_order_line": mx(d_lin), "network": mx(d_net)},
               "network_over_constant_rms": round(rms(d_net) / rms(d_const), 4)}
        log("residual step %g: held-out RMS plain %.4f, constant %.4f, first-order line %.4f, network %.4f mHa"
            % (step_sigma, rms(d_plain), rms(d_const), rms(d_lin), rms(d_net)))
        if step_sigma == step_sigmas[0]:
            est = RES.CorrectedLO(ctx, f, lbar, model, bound_mha=0.2, check_every=10, check_walkers=64,
                                  reference=exact)
            th = theta   # the last step of every walk
            est(th)   # first call checks
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            reps = 20
            e0.record()
            for _ in range(reps):
                est(th)
            e1.record()
            torch.cuda.synchronize()
            rec["check"] = est.last_check
            rec["corrected_lo_ms_per_call"] = round(e0.elapsed_time(e1) / reps, 3)
        out["walks"]["%g" % step_sigma] = rec
        del x, ef, el, xtr, xte
    f.close()
    ctx.close()
    return out


def md_study(torch, lofqmc, synth, steps, warmup, baseline_steps=2):
    """Multi-determinant trial on the 400-site CAS chain (60 occupied + 5 active
    virtual orbitals, 5 active occupied, 200 determinants up to quadruples, 512
    walkers, LO at 1e-5): reference green_theta + local_energy_md per step (the
    SMW route of Eq. 20-23), against evaluating every determinant on its own
    (green_theta with that determinant and the LO energy over the padded n_cas
    orbitals, weighted by c_d det^2), which also cross-checks the energies."""
    cfg = synth.CAS_POLYACENE
    log("multi-determinant study: generating %s" % cfg.name)
    s = synth.make_cas_system(cfg)
    M, n, nw, ncas, ndet = cfg.M, cfg.n, cfg.nw, cfg.n_cas, cfg.n_det
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    ctx = lofqmc.Context()
    C, ref, phi = dev(s.orbitals), dev(s.reference), dev(s.walkers)
    lbar = ctx.build_half_rotated_chol(dev(s.chol), C)
    t0 = time.perf_counter()
    f = ctx.build_lo_factors(lbar, cfg.epsilon)
    md = ctx.build_md_trial(f, n, cfg.n_act_occ, C, s.holes, s.particles, s.coeffs)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    theta = torch.empty((nw, n, M), dtype=torch.complex128, device="cuda")   # transposed, as the LO step
    logov = torch.empty(nw, dtype=torch.complex128, device="cuda")
    info = torch.empty(nw, dtype=torch.int32, device="cuda")
    energy = torch.empty((nw, 2), dtype=torch.complex128, device="cuda")
    ovr = torch.empty(nw, dtype=torch.complex128, device="cuda")

    def step(ev):
        if ev is not None:
            ev["a"].record()
        ctx.green_theta(ref, phi, theta, logov, info, transposed=True)
        if ev is not None:
            ev["b"].record()
        ctx.local_energy_md(md, theta, info, energy, ovr, transposed=True)
        if ev is not None:
            ev["c"].record()

    tot, split, kern = time_route(torch, ctx, step, steps, warmup, ["a", "b", "c"])
    ms = tot / steps
    e_md = energy.cpu().numpy()
    log("multi-determinant: %.3f ms/step (local_energy_md %.3f), %d determinants, %d pairs"
        % (ms, float(np.mean(split["b->c"])), ndet, md.npairs))

    # every determinant on its own
    trials, occs = [], []
    for h, p in zip(s.holes, s.particles):
        occ = list(range(n))
        for a, b in zip(h, p):
            occ[a] = b
        occs.append(torch.tensor(occ, dtype=torch.int64, device="cuda"))
        trials.append(C[:, occs[-1]].contiguous())
    coef = torch.tensor(s.coeffs, dtype=torch.complex128, device="cuda")
    th_d = torch.empty((nw, M, n), dtype=torch.complex128, device="cuda")
    lo_d = torch.empty(nw, dtype=torch.complex128, device="cuda")
    inf_d = torch.empty(nw, dtype=torch.int32, device="cuda")
    pad = torch.zeros((nw, M, ncas), dtype=torch.complex128, device="cuda")
    e_d = torch.empty((nw, 2), dtype=torch.complex128, device="cuda")

    def per_det():
        num = torch.zeros((nw, 2), dtype=torch.complex128, device="cuda")
        den = torch.zeros(nw, dtype=torch.complex128, device="cuda")
        for d in range(ndet):
            ctx.green_theta(trials[d], phi, th_d, lo_d, inf_d)
            pad.zero_()
            pad[:, :, occs[d]] = th_d
            ctx.local_energy_lo(f, pad, inf_d, energy=e_d)
            ov = coef[d] * torch.exp(2.0 * (lo_d - logov))
            num += ov[:, None] * e_d
            den += ov
        return num / den[:, None]

    e_pd = per_det()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(baseline_steps):
        per_det()
    t1.record()
    torch.cuda.synchronize()
    pd_ms = t0.elapsed_time(t1) / baseline_steps + float(np.mean(split["a->b"]))
    diff = float(np.abs(e_md - e_pd.cpu().numpy()).max())
    log("per-determinant evaluation: %.1f ms/step, max |E_md - E_per_det| %.2e Ha" % (pd_ms, diff))
    own = [k for k in kern if k.startswith("md_") or k == "lo_pass1_kernel" or k == "reduce_partials_kernel"]
    # algorithmic work per launch (unpadded sizes): pass 1 as in the single-
    # determinant route; md_prep: T = C_av^T theta, a Gauss-Jordan inverse of
    # every eps_d x eps_d R_d and its eps_d^4 moment products, then Y_o =
    # Omega tau_o for every orbital (n_cas nao^2 nav^2 products); md_energy:
    # per pair and rank row the own products, the four mean projections and
    # the outer product G, then M = Y_i tau_j (nao^2 nav) and two nao^2 forms
    nao, nav = cfg.n_act_occ, cfg.n_act_virt
    finfo = f.info()
    ranks = finfo["ranks"]
    iu = np.triu_indices(ncas)
    Ks = ranks[iu][ranks[iu] > 0].astype(np.float64)
    eps_d = np.array([len(h) for h in s.holes], dtype=np.float64)
    mdwork = {
        "lo_pass1_kernel": ("mfma", 4.0 * M * md.out_rows * nw,
                            8.0 * M * finfo["total_rows"] + 16.0 * nw * (M * n + md.out_rows)),
        "md_prep_kernel": ("alu", nw * (4.0 * M * nav * n + np.sum(8.0 * eps_d ** 3 + 16.0 * eps_d ** 4)
                                        + 8.0 * ncas * nao * nao * nav * nav),
                           16.0 * nw * (M * n + nao * nav * (1 + nao * nav) + ncas * nao * nao * nav)),
        "md_energy_kernel": ("alu", nw * 8.0 * float(np.sum(Ks * (2 + 4 * nao + nao * nao)
                                                           + nao * nao * nav + 2 * nao * nao)),
                             16.0 * nw * md.out_rows),
    }
    md_roof = {k: roofline_of(k, mdwork, kern[k][1] / kern[k][0]) for k in mdwork if k in kern}
    out = {"workload": cfg.name, "M": M, "n_occ": n, "n_cas": ncas, "n_act_occ": cfg.n_act_occ,
           "n_act_virt": cfg.n_act_virt, "n_det": ndet, "max_exc": cfg.max_exc, "walkers": nw,
           "epsilon": cfg.epsilon, "n_chol": s.chol.shape[0], "setup_s": round(setup_s, 2),
           "value": round(nw / (ms * 1e-3), 1), "unit": "walker-energies/s", "ms_per_step": round(ms, 4),
           "local_energy_md_ms": round(float(np.mean(split["b->c"])), 4),
           "kernel_us": {k: round(kern[k][1] / kern[k][0] * 1e3, 2) for k in own},
           "kernels": md_roof,
           "pass1_out_rows": md.out_rows, "pairs": md.npairs,
           "per_determinant_ms_per_step": round(pd_ms, 2),
           "smw_speedup_vs_per_determinant": round(pd_ms / ms, 1),
           "max_abs_diff_vs_per_determinant_Ha": diff}
    # cost against the number of determinants (same walkers and factors; every
    # excitation up to quadruples: 250 besides the reference)
    scaling = []
    for k in (1, 20, 100, 251):
        h, p_, c = synth.cas_expansion(n, cfg.n_act_occ, cfg.n_act_virt, k, cfg.max_exc, np.random.default_rng(k))
        mk = ctx.build_md_trial(f, n, cfg.n_act_occ, C, h, p_, c)
        ms_k = event_ms(torch, lambda mk=mk: ctx.local_energy_md(mk, theta, info, energy, transposed=True))
        scaling.append({"n_det": k, "local_energy_md_ms": round(ms_k, 4)})
        mk.close()
    out["n_det_scaling"] = scaling
    log("local_energy_md vs determinants: %s" % ", ".join("%d: %.3f ms" % (x["n_det"], x["local_energy_md_ms"])
                                                         for x in scaling))
    md.close()
    f.close()
    ctx.close()
    return out


def cpu_baseline(cfg, system, eps, sample):
    """The CPU reference (numpy FP64) on a fixed sample of walkers: LO route."""
    from oracle import energy as E
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [os.cpu_count()])
    except Exception:
        threads = os.cpu_count()
    lbar = E.half_rotate(system.chol, system.trial)
    log("cpu baseline: SVD compression of %d pair blocks (set-up, untimed)" % (cfg.n * (cfg.n + 1) // 2))
    fac = E.lo_compress(lbar, eps, pairs="upper")
    walkers = system.walkers[:sample]
    t = time.perf_counter()
    for phi in walkers:
        theta, _, _ = E.green_theta(system.trial, phi)
        E.e2_lo(fac, theta)
    dt = time.perf_counter() - t
    return {"value": sample / dt, "unit": "walker-energies/s", "cores": int(threads), "kind": "oracle",
            "sample": "LO route (green_theta + LO energy) of the first %d of %d walkers at eps=%g, %.1f s"
                      % (sample, cfg.nw, eps, dt)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=400)
    ap.add_argument("--cpu-sample", type=int, default=256,
                    help="walkers timed on the CPU reference (about 10 s of host work at the default)")
    ap.add_argument("--eps", type=str, default="",
                    help="comma-separated LO thresholds to run instead of the workload's sweep")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the reduced-precision study on the 500-site chain")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the multi-system batching study (8 chain systems, captured graph)")
    ap.add_argument("--no-residual", action="store_true",
                    help="skip the learned-residual study (800-site chain: about 30 GB of device memory)")
    ap.add_argument("--no-md", action="store_true", help="skip the multi-determinant study")
    ap.add_argument("--no-wm", action="store_true",
                    help="skip the headline step with walker-major theta (counter runs: every pass-1 launch of "
                         "the LO route then reads transposed theta)")
    ap.add_argument("--no-hr", action="store_true",
                    help="skip the half-rotated ERI route (Eq. 17; its pair blocks take 2.3 GB)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run one plain device copy of this size (HBM counter calibration)")
    ap.add_argument("--traffic-table", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="only write profiles/hbm_traffic.json from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs of "
                         "this bench (one threshold, --eps) and of --calibrate-copy-mib 1024; no GPU needed")
    args = ap.parse_args()
    if args.traffic_table:
        eps = float(args.eps) if args.eps else EPS_SWEEP[0]
        t = write_traffic_table(*args.traffic_table, eps, "chain-M400-n60-w512",
                                os.path.join(ROOT, "profiles", "hbm_traffic.json"))
        for k, v in t["kernels"].items():
            for ln in v["launches"]:
                print("%-24s grid %9d  read %8.1f MB  write %8.1f MB" % (k, ln["grid"], ln["read_bytes"] / 1e6,
                                                                          ln["write_bytes"] / 1e6))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the walker batch of this workload is a single GPU's share, "
              "and no multi-GPU path is built (got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib * (1 << 20) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8}))
        return

    from paper_2202_00832_amd import lofqmc, synth

    cfg = synth.CHAIN_POLYACENE
    log("generating %s" % cfg.name)
    system = synth.make_system(cfg)
    M, n, nw, X = cfg.M, cfg.n, cfg.nw, system.n_chol
    log("M=%d n=%d X=%d walkers=%d" % (M, n, X, nw))

    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    chol_d, trial_d, phi_d = dev(system.chol), dev(system.trial), dev(system.walkers)
    ctx = lofqmc.Context()
    t = time.perf_counter()
    lbar = ctx.build_half_rotated_chol(chol_d, trial_d)
    torch.cuda.synchronize()
    t_half = time.perf_counter() - t
    del chol_d
    log("half-rotation %.2f s" % t_half)

    theta, logov, info = ctx.green_theta(trial_d, phi_d)
    e_full = ctx.local_energy_full(lbar, theta, info)
    # the LO route reads theta transposed ([w][j][r]), in the accuracy sweep too
    theta_tr, _, _ = ctx.green_theta(trial_d, phi_d, transposed=True)
    torch.cuda.synchronize()
    assert int((info != 0).sum()) == 0, "singular walker overlap"
    e_full_h = e_full.cpu().numpy()
    E2_full = e_full_h.sum(axis=1)

    sweep = []
    factors = {}
    epsilons = [float(e) for e in args.eps.split(",")] if args.eps else list(EPS_SWEEP)
    for eps in epsilons:
        t = time.perf_counter()
        f = ctx.build_lo_factors(lbar, eps)
        t_build = time.perf_counter() - t
        factors[eps] = f
        e_lo = ctx.local_energy_lo(f, theta_tr, info, transposed=True)
        torch.cuda.synchronize()
        E2_lo = e_lo.cpu().numpy().sum(axis=1)
        dre = (E2_lo - E2_full).real
        d = np.abs(dre)
        mean_err = abs(dre.mean()) + 2.0 * dre.std(ddof=1) / np.sqrt(nw)
        inf = f.info()
        ranks = inf["ranks"]
        sweep.append({"epsilon": eps, "build_s": round(t_build, 3), "mean_rank": float(ranks.mean()),
                      "max_rank": int(ranks.max()),
                      "compression_pct": float(100.0 * (M - ranks.mean()) / M),
                      "factor_mib": inf["bytes"] / 2 ** 20,
                      "max_abs_dE_mHa": float(d.max() * 1e3), "mean_dE_mHa": float((E2_lo - E2_full).real.mean() * 1e3),
                      "sd_dE_mHa": float((E2_lo - E2_full).real.std() * 1e3),
                      "p99_abs_dE_mHa": float(np.percentile(d, 99) * 1e3),
                      "total_energy_err_bound_mHa": float(mean_err * 1e3),
                      "passes_1mHa_per_walker": bool(d.max() <= GATE_HA),
                      "passes_1mHa_mean": bool(mean_err <= GATE_HA),
                      # algorithmic pass-1 output rows 4 sum_{i<j} K_ij + sum_i K_ii and
                      # factor rows 2 sum_{i<j} K_ij + sum_i K_ii (ranks is the ordered n x n table)
                      "_n_out": int(2 * ranks.sum() - np.trace(ranks)), "_total_rows": int(ranks.sum()),
                      "_pair_rows": int((ranks.sum() + np.trace(ranks)) // 2)})
        log("eps=%g: build %.1f s, <K>=%.3f, total-energy error <= %.3f mHa, max per-walker |dE| %.3e mHa"
            % (eps, t_build, ranks.mean(), mean_err * 1e3, d.max() * 1e3))
    def pick(key):
        passing = [s for s in sweep if s[key]]
        return max(passing, key=lambda s: s["epsilon"]) if passing else min(sweep, key=lambda s: s["epsilon"])
    head = pick("passes_1mHa_per_walker")
    head_mean = pick("passes_1mHa_mean")
    eps_h = head["epsilon"]

    energy = torch.empty((nw, 2), dtype=torch.complex128, device="cuda")
    # the LO step hands theta over transposed ([w][j][r], theta_tr), the
    # layout whose orbital columns pass 1 loads in whole cache lines (same
    # energies bit for bit as walker-major theta)

    def lo_step_for(f):
        def step(ev):
            if ev is not None:
                ev["a"].record()
            ctx.green_theta(trial_d, phi_d, theta_tr, logov, info, transposed=True)
            if ev is not None:
                ev["b"].record()
            ctx.local_energy_lo(f, theta_tr, info, energy, transposed=True)
            if ev is not None:
                ev["c"].record()
        return step

    def full_step(ev):
        if ev is not None:
            ev["a"].record()
        ctx.green_theta(trial_d, phi_d, theta, logov, info)
        if ev is not None:
            ev["b"].record()
        ctx.local_energy_full(lbar, theta, info, energy)
        if ev is not None:
            ev["c"].record()

    marks = ["a", "b", "c"]
    results = {}
    for s in sweep:
        tot, split, kern = time_route(torch, ctx, lo_step_for(factors[s["epsilon"]]), args.steps, args.warmup,
                                      marks)
        s["_kernels"] = kern
        s["kernel_us"] = {k: round(t / c * 1e3, 2) for k, (c, t) in kern.items()}
        s["ms_per_step"] = tot / args.steps
        s["walker_energies_per_s"] = nw / (tot / args.steps / 1e3)
        s["green_theta_ms"] = float(np.mean(split["a->b"]))
        s["local_energy_lo_ms"] = float(np.mean(split["b->c"]))
        results[s["epsilon"]] = split
        log("LO eps=%g: %.3f ms/step (green_theta %.3f, LO %.3f)" % (s["epsilon"], s["ms_per_step"],
                                                                     s["green_theta_ms"], s["local_energy_lo_ms"]))
    # the headline step again with walker-major theta ([w][r][j]), for the
    # layout comparison (same energies bit for bit)
    def lo_step_wm(ev):
        if ev is not None:
            ev["a"].record()
        ctx.green_theta(trial_d, phi_d, theta, logov, info)
        if ev is not None:
            ev["b"].record()
        ctx.local_energy_lo(factors[head_eps], theta, info, energy)
        if ev is not None:
            ev["c"].record()
    head_eps = head["epsilon"]
    lo_wm = None
    if not args.no_wm:
        tot_w, _, kern_w = time_route(torch, ctx, lo_step_wm, args.steps, min(args.warmup, 50), marks)
        lo_wm = {"epsilon": head_eps, "ms_per_step": round(tot_w / args.steps, 4),
                 "walker_energies_per_s": round(nw / (tot_w / args.steps / 1e3), 1),
                 "kernel_us": {k: round(t / c * 1e3, 2) for k, (c, t) in kern_w.items()}}
        log("LO eps=%g, walker-major theta: %.3f ms/step" % (head_eps, lo_wm["ms_per_step"]))
    full_steps = max(1, min(args.steps, 10))
    tot_f, split_f, kern_f = time_route(torch, ctx, full_step, full_steps, min(args.warmup, 2), marks)
    full_ms = tot_f / full_steps
    full_energy_ms = float(np.mean(split_f["b->c"]))
    log("full: %.3f ms/step (local_energy_full %.3f)" % (full_ms, full_energy_ms))

    # roofline of the dominant kernel of the headline step (largest summed
    # duration in the timed region), from the library's per-kernel events
    work = kernel_work(M, n, nw, X, head["_n_out"], head["_total_rows"], head["_pair_rows"])
    kern = head["_kernels"]
    per_kernel = {k: roofline_of(k, work, t / c) for k, (c, t) in kern.items() if k in work}
    dom = max(kern, key=lambda k: kern[k][1])
    roofline = dict(per_kernel[dom])
    tr = measured_traffic(dom, head["epsilon"])
    roofline["traffic"] = round(tr) if tr is not None else None
    full_kernels = {k: roofline_of(k, work, t / c) for k, (c, t) in kern_f.items() if k in work}
    full_roof = full_kernels["energy_full_kernel"]

    hr_out = None
    if not args.no_hr:
        hr_out = hr_study(torch, ctx, lbar, trial_d, phi_d, info, energy, e_full_h, work, M, n, nw)
        # the paper's comparison (Sec. 3, dodecane): LO against the HR-ERI
        # energy evaluation at each threshold, energy call alone and whole step
        hr_out["walkers16"] = few_walker_study(torch, ctx, lbar, trial_d, phi_d, factors)
        hr_out["lo_speedup"] = {
            "%g" % s["epsilon"]: {"energy_only": round(hr_out["local_energy_hr_ms"] / s["local_energy_lo_ms"], 1),
                                  "step": round(hr_out["ms_per_step"] / s["ms_per_step"], 1)} for s in sweep}

    prec = None
    if not args.no_precision:
        release_cached(torch, "precision study")
        prec = precision_study(torch, lofqmc, synth, max(2, min(args.steps, 5)))
    batch = None
    if not args.no_batch:
        release_cached(torch, "batching study")
        batch = batch_study(torch, lofqmc, synth)
    mdet = None
    if not args.no_md:
        release_cached(torch, "multi-determinant study")
        mdet = md_study(torch, lofqmc, synth, max(5, min(args.steps, 50)), min(args.warmup, 20))
    resid = None
    if not args.no_residual:
        release_cached(torch, "residual study")
        resid = residual_study(torch, lofqmc, synth)

    log("CPU reference baseline (%d walkers)" % args.cpu_sample)
    cpu = cpu_baseline(cfg, system, eps_h, args.cpu_sample)
    log("cpu: %.2f walker-energies/s" % cpu["value"])

    value = head["walker_energies_per_s"]
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "walker-energies/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg.name, "M": M, "n_occ": n, "n_chol": X, "walkers": nw, "sigma": cfg.sigma,
                   "cholesky_tol": cfg.chol_tol, "route": "LO", "epsilon": eps_h,
                   "theta_layout": "[w][j][r] (each walker's theta transposed)",
                   "gate": "max over walkers of |Re(E_LO - E_full)| <= 1 mHa"},
        "lo_walker_major_theta": lo_wm,
        "value_mean_gate": {"value": round(head_mean["walker_energies_per_s"], 1), "unit": "walker-energies/s",
                            "epsilon": head_mean["epsilon"],
                            "gate": "|mean Re(E_LO - E_full)| + 2 stderr <= 1 mHa over the walkers"},
        "full": {"value": round(nw / (full_ms * 1e-3), 1), "unit": "walker-energies/s", "ms_per_step": round(full_ms, 4),
                 "steps": full_steps, "roofline": full_roof, "kernels": full_kernels},
        "lo_vs_full_speedup": round(full_ms / head["ms_per_step"], 2),
        "hr_eri": hr_out,
        "eps_sweep": [{k: v for k, v in s.items() if not k.startswith("_")} for s in sweep],
        "roofline": roofline,
        "kernels": per_kernel,
        "mixed_precision": prec,
        "batching": batch,
        "multi_determinant": mdet,
        "learned_residual": resid,
        "cpu_baseline": cpu,
        "setup_s": {"half_rotation": round(t_half, 3)},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
