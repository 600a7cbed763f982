#!/usr/bin/env python
"""Throughput of the chi0 application (one step = chi0bar applied to the seeded block
of N_pdep trial potentials: N_pdep * N_v Sternheimer solves to tolerance, density
response and Coulomb-scaled projection) on one MI355X.

Default workload "medium": 20^3 bohr cell, 48^3 grid, 12 Ha (15895 plane waves),
64 Gaussian wells, N_v = 128, N_pdep = 128 (16384 Sternheimer systems per step),
mixed precision (FP32 inner CG, FP64 refinement to 1e-8), inputs resident in HBM.
The FP64 path is timed on the same block for the speedup, and the mixed result counts
only if its Rayleigh-Ritz dielectric eigenvalues on the block agree with the FP64
path's within 1e-6.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6, "bf16": 2500.0}
VECTOR_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
# kernel classes whose algorithmic flops run on the vector ALUs (FFT arithmetic); the
# others that report flops run on the matrix cores
VALU_KERNELS = {"slab_hv": "f32", "slab_hv_fp64": "f64"}
# Measured HBM traffic of a kernel class, KiB per dispatch averaged over one bench step of
# the medium workload: rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE, scaled by the factors
# that make a plain 1 GiB copy (torch.mul) read and write 1 GiB (2.0 and 1.0).  Reported
# only while the kernel source file is the one that was measured.
MEASURED_TRAFFIC = {
    "slab_hv": {"fetch_kib": 64999.8, "write_kib": 125397.0, "fetch_scale": 2.0, "write_scale": 1.0,
                "source": "paper_1501_03141_amd/csrc/fft.hip", "sha1": "431bb546f434d0e912ea35467b6b21204735f839",
                "workload": "medium"},
}


def measured_traffic(name: str, workload: str):
    """HBM bytes per launch from the committed counter runs, or None."""
    import hashlib
    m = MEASURED_TRAFFIC.get(name)
    if m is None or m["workload"] != workload:
        return None
    try:
        with open(os.path.join(ROOT, m["source"]), "rb") as f:
            if hashlib.sha1(f.read()).hexdigest() != m["sha1"]:
                return None
    except OSError:
        return None
    return 1024.0 * (m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"])


def ritz_eps(phi: np.ndarray, chi_phi: np.ndarray) -> np.ndarray:
    """Dielectric eigenvalues 1 - theta of chi0bar projected on span(phi) (real
    coefficients; phi rows Hermitian-symmetric)."""
    import scipy.linalg as sla
    S = np.real(phi.conj() @ phi.T)
    M = np.real(phi.conj() @ chi_phi.T)
    M = 0.5 * (M + M.T)
    th = sla.eigh(M, S, eigvals_only=True)
    return np.sort(1.0 - th)[::-1]


def make_context(w, V, precision, psi=None, eps=None, **kw):
    from paper_1501_03141_amd import pdep
    return pdep.Context(w.L, w.n, w.ecut, V, w.n_v, precision=precision, cg_tol=w.cg_tol,
                        psi=psi, eps=eps, device_ptrs=True, **kw)


def dominant_roofline(prof: dict, mfma_dtype: str):
    """Roofline object for the kernel class with the largest device time.  Matrix-core
    kernels are priced at the dense peak of the type they run on (bf16 for the BF16x3
    split, whose three products per product cap algorithmic flops at a third of it)."""
    name, rec = max(prof.items(), key=lambda kv: kv[1]["ms"])
    t = rec["ms"] / 1e3
    if rec["flops"] > 0 and name in VALU_KERNELS:
        # FFT arithmetic bounds this kernel: its vector-ALU floor lies above its HBM floor
        ach = rec["flops"] / t / 1e12
        peak = VECTOR_PEAK_TFLOPS[VALU_KERNELS[name]]
        return name, {"bound": "alu", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
                      "frac": round(ach / peak, 4), "traffic": None,
                      "hbm_achieved_gbs": round(rec["bytes"] / t / 1e9, 1),
                      "avg_launch_ms": round(rec["ms"] / max(rec["launches"], 1), 4),
                      "launches": rec["launches"]}
    if rec["flops"] > 0:
        if name.endswith("_fp64"):
            mfma_dtype = "f64"
        ach = rec["flops"] / t / 1e12
        peak = MFMA_PEAK_TFLOPS[mfma_dtype]
        r = {"bound": "mfma", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
             "frac": round(ach / peak, 4), "traffic": None,
             "avg_launch_ms": round(rec["ms"] / max(rec["launches"], 1), 4), "launches": rec["launches"]}
        if mfma_dtype == "bf16":
            r["peak_algorithmic_bf16x3"] = round(peak / 3, 1)
        return name, r
    ach = rec["bytes"] / t / 1e9
    return name, {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                  "avg_launch_ms": round(rec["ms"] / max(rec["launches"], 1), 4),
                  "launches": rec["launches"]}


def cpu_baseline(w, V, eps, psi, phi_host, n_bands: int):
    """The CPU FP64 oracle (matrix-free FFT + CG) on a bounded sample: one
    perturbation, n_bands occupied bands spread evenly over the occupied range (low
    bands converge in few iterations, bands next to the gap in many).  Returns apps/s
    extrapolated to all N_v bands (time per Sternheimer system x N_v)."""
    from oracle import matfree as MF
    from oracle import response as R
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    m = R.make_model(w.L, w.n, w.ecut, V, naive=False)
    gs = R.GroundState(np.asarray(eps), np.asarray(psi), m.inv(np.asarray(psi)), 0.0)
    sel = np.unique(np.linspace(0, w.n_v - 1, n_bands).round().astype(int))
    t0 = time.perf_counter()
    _, iters = MF.chi0bar_apply_cg(m, gs, phi_host[:1], w.cg_tol, bands=sel)
    dt = time.perf_counter() - t0
    per_system = dt / len(sel)
    apps = 1.0 / (per_system * w.n_v)
    return {"value": apps, "unit": "applications/s", "cores": int(cores), "kind": "oracle",
            "sample": f"1 perturbation x {len(sel)} of {w.n_v} bands evenly spaced (FP64 FFT+CG oracle, "
                      f"{iters} CG iterations in total, {dt:.1f} s), extrapolated per Sternheimer system "
                      f"to all {w.n_v} bands",
            "seconds": round(dt, 2)}


def serving_bench(n_jobs: int, max_running: int, log):
    """Serving stream of the shape of the paper-scale job mix (grids 24^3/32^3/48^3,
    N_v 8..128, N_pdep 16..64, wells scaled with the cell volume).  Phase 1 submits all
    jobs at once to measure capacity (jobs/s); phase 2 replays the stream with Poisson
    arrivals at 0.8 x capacity and reports latency percentiles."""
    from paper_1501_03141_amd import inputs, pdep

    def run(jobs, arrivals):
        lat, ok = [], 0
        with pdep.Server(max_running=max_running) as srv:
            t0 = time.perf_counter()
            tickets = []
            for job, ta in zip(jobs, arrivals):
                dt = ta - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                w = job.workload
                tickets.append(srv.submit(w.L, w.n, w.ecut, inputs.vloc(w), w.n_v, w.n_pdep, seed=w.seed,
                                          precision=pdep.PDEP_MIXED_FP32, cg_tol=1e-8, eig_tol=1e-6,
                                          eig_maxit=60, n_buffer=8, gap_min=1e-4))
            for job, t in zip(jobs, tickets):
                srv.wait(t, -1)
                state, res, _ = srv.poll(t)
                if state == pdep.JOB_DONE:
                    ok += 1
                    lat.append(res["latency_ms"])
                else:
                    w = job.workload
                    log(f"  job {w.name} grid {w.n[0]} N_v {w.n_v} N_pdep {w.n_pdep} failed: "
                        f"{res.get('error')} ({res['run_ms']:.0f} ms)")
            wall = time.perf_counter() - t0
            peak = srv.stats()["peak_running"]
        return wall, lat, ok, peak

    jobs = inputs.serving_stream(n_jobs, rate_hz=1.0)
    wall, lat, ok, peak = run(jobs, [0.0] * len(jobs))
    capacity = ok / wall
    log(f"serving burst: {ok}/{len(jobs)} jobs in {wall:.1f} s -> capacity {capacity:.2f} jobs/s")
    rate = 0.8 * capacity
    jobs2 = inputs.serving_stream(n_jobs, rate_hz=rate, base_seed=2506)
    arrivals = [j.arrival_s - jobs2[0].arrival_s for j in jobs2]
    wall2, lat2, ok2, peak2 = run(jobs2, arrivals)
    log(f"serving stream at {rate:.2f} jobs/s: {ok2}/{len(jobs2)} done in {wall2:.1f} s")
    return {"jobs": n_jobs, "max_running": max_running, "capacity_jobs_per_s": round(capacity, 3),
            "offered_rate_jobs_per_s": round(rate, 3), "jobs_per_s": round(ok2 / wall2, 3),
            "p50_ms": round(float(np.percentile(lat2, 50)), 1) if lat2 else None,
            "p99_ms": round(float(np.percentile(lat2, 99)), 1) if lat2 else None,
            "failed": len(jobs2) - ok2, "peak_running": peak2,
            "sample": f"{n_jobs}-job Poisson stream (grids 24^3/32^3/48^3, N_v 8..128, N_pdep 16..64), "
                      "mixed precision, Davidson to 1e-6 with 8 buffer vectors"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="medium")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-bands", type=int, default=48)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--precision", choices=["bf16x3", "mixed_fp32"], default="bf16x3",
                    help="mixed mode of the timed steps (the other one is timed once beside it)")
    ap.add_argument("--no-other-mode", action="store_true")
    ap.add_argument("--no-eigs", action="store_true", help="skip the end-to-end PDEP Davidson")
    ap.add_argument("--serving-jobs", type=int, default=24, help="0 disables the serving phase")
    ap.add_argument("--serving-max-running", type=int, default=4)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the timed steps, copy a buffer of this size 3 times (reference "
                         "kernel for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path would shard by "
              "perturbation across GPUs, which this benchmark does not run.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1501_03141_amd import inputs, pdep

    torch.cuda.set_device(0)
    w0 = inputs.WORKLOADS[args.workload]
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731

    # ---- setup (excluded from the metric): ground state on the GPU, seed advanced on EGAP
    t_setup = time.perf_counter()
    ctx = None
    for k in range(8):
        w = inputs.with_seed(w0, w0.seed + k)
        V = inputs.vloc(w)
        try:
            ctx = make_context(w, V, pdep.PDEP_MIXED_FP32, gs_tol=1e-10)
            break
        except pdep.PdepError as e:
            if e.code != pdep.PDEP_EGAP:
                raise
            log(f"seed {w.seed}: {e}; advancing seed")
    assert ctx is not None
    setup_s = time.perf_counter() - t_setup
    log(f"setup {setup_s:.1f} s: n_pw {ctx.n_pw}, gap {ctx.gap:.4f} Ha, gs iters {ctx.gs_iterations}, "
        f"gs residual {ctx.gs_residual:.2e}")
    miller = ctx.miller()
    nz = np.any(miller != 0, axis=1)
    phi_host = inputs.trial_block(miller[nz], w.n_pdep, w.seed)
    phi = torch.from_numpy(phi_host).cuda()
    out = torch.empty_like(phi)
    eps_occ, psi = ctx.orbitals()

    modes = {"mixed_fp32": pdep.PDEP_MIXED_FP32, "bf16x3": pdep.PDEP_MIXED_BF16X3}
    main_mode = args.precision
    other_mode = "mixed_fp32" if main_mode == "bf16x3" else "bf16x3"
    ctx_main = ctx if main_mode == "mixed_fp32" else make_context(w, V, modes[main_mode], psi=psi, eps=eps_occ)

    def run_steps(c, o, steps, warmup, profile, classes=None):
        """profile: time kernel launches with events (classes: only those classes)."""
        for _ in range(warmup):
            _, st = c.chi0_apply(phi, out=o)
            log("warmup", st)
        torch.cuda.synchronize()
        if profile:
            pdep.profile_classes(classes)
            pdep.profile_read(reset=True)
            pdep.profile_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = []
        for _ in range(steps):
            _, st = c.chi0_apply(phi, out=o)
            sts.append(st)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pr = None
        if profile:
            pdep.profile_enable(False)
            pr = pdep.profile_read(reset=True)
        return (t1 - t0) * 1e3 / steps, sts, pr

    # ---- warmup, one untimed step with every launch timed (kernel breakdown), then the
    # timed steps with live events on the dominant kernel class only
    _, _, prof = run_steps(ctx_main, out, 1, args.warmup, True)
    for kname, rec in sorted(prof.items(), key=lambda kv: -kv[1]["ms"]):
        if rec["launches"]:
            log(f"  {kname:20s} {rec['ms']:10.2f} ms  {rec['launches']:7d} launches  "
                f"{rec['bytes'] / max(rec['ms'], 1e-9) / 1e6:8.1f} GB/s  {rec['flops'] / max(rec['ms'], 1e-9) / 1e9:8.2f} TF/s")
    dominant = max(prof.items(), key=lambda kv: kv[1]["ms"])[0]
    ms_step, stats, prof_dom = run_steps(ctx_main, out, args.steps, 0, True, classes=[dominant])
    value = w.n_pdep / (ms_step / 1e3)
    chi_mixed = out.cpu().numpy()
    log(f"timed ({main_mode})", stats[-1], f"{ms_step:.1f} ms/step")
    kname, roof = dominant_roofline({dominant: prof_dom[dominant]}, "bf16" if main_mode == "bf16x3" else "f32")
    pdep.profile_classes(None)
    roof["traffic"] = measured_traffic(kname, w0.name)
    if roof["traffic"] is not None:
        roof["traffic_unit"] = "bytes/launch"
        roof["algorithmic_bytes_per_launch"] = round(prof_dom[kname]["bytes"] / max(prof_dom[kname]["launches"], 1))
    if args.copy_probe_mib > 0:
        src = torch.empty(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)     # one elementwise kernel: N bytes read, N written
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written per copy")
        del src, dst

    # ---- FP64 path on the same block (speedup and the 1e-6 eigenvalue check)
    fp64 = None
    eps_err = None
    other = None
    if not args.no_fp64:
        ctx64 = make_context(w, V, pdep.PDEP_FP64, psi=psi, eps=eps_occ)
        out64 = torch.empty_like(phi)
        ms64, sts64, _ = run_steps(ctx64, out64, 1, 1, False)
        st64 = sts64[-1]
        chi64 = out64.cpu().numpy()
        e_fp64 = ritz_eps(phi_host, chi64)
        eps_err = float(np.max(np.abs(ritz_eps(phi_host, chi_mixed) - e_fp64)))
        fp64 = {"ms_per_step": round(ms64, 2), "value": round(w.n_pdep / (ms64 / 1e3), 3),
                "fft_chunk_rows": st64["fft_chunk"],
                "cg_iter_max": st64["cg_iter_max"], "speedup_mixed_over_fp64": round(ms64 / ms_step, 3)}
        log("fp64", st64, f"{ms64:.1f} ms; ritz eps err {main_mode} vs fp64 {eps_err:.2e}")
        ctx64.close()
        # the other mixed mode, one warm-up and one timed step
        if not args.no_other_mode:
            ctx_o = ctx if other_mode == "mixed_fp32" else make_context(w, V, modes[other_mode], psi=psi, eps=eps_occ)
            out_o = torch.empty_like(phi)
            ms_o, sts_o, _ = run_steps(ctx_o, out_o, 1, 1, False)
            err_o = float(np.max(np.abs(ritz_eps(phi_host, out_o.cpu().numpy()) - e_fp64)))
            other = {"precision": other_mode, "ms_per_step": round(ms_o, 2),
                     "value": round(w.n_pdep / (ms_o / 1e3), 3), "eps_err_vs_fp64": err_o,
                     "cg_iter_max": sts_o[-1]["cg_iter_max"], "refine_steps": sts_o[-1]["refine_steps"]}
            log(f"{other_mode}", sts_o[-1], f"{ms_o:.1f} ms; ritz eps err vs fp64 {err_o:.2e}")
            if ctx_o is not ctx:
                ctx_o.close()

    # ---- end-to-end PDEP: block Davidson for the N_pdep most screened eigenpairs from the
    # library's own random start (main mixed mode)
    eigs = None
    if not args.no_eigs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eps_pdep, _, est = ctx_main.eigs(w.n_pdep, seed=w.seed, tol=1e-6, maxit=60, n_buffer=8, allow_notconv=True)
        torch.cuda.synchronize()
        t_e = time.perf_counter() - t0
        eigs = {"seconds": round(t_e, 2), "n_pdep": w.n_pdep, "tol": 1e-6, "n_buffer": 8,
                "iterations": est["iterations"], "chi0_columns": est["chi0_columns"],
                "max_residual": est["max_residual"], "eps_max": float(eps_pdep[0]),
                "eps_min": float(eps_pdep[-1])}
        log("pdep_eigs", eigs)

    serving = None
    if args.serving_jobs > 0:
        serving = serving_bench(args.serving_jobs, args.serving_max_running, log)
        log("serving", serving)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, V, eps_occ, psi, phi_host, min(args.cpu_bands, w.n_v))
        log("cpu baseline", cpu)
    if ctx_main is not ctx:
        ctx_main.close()
    ctx.close()

    rec = {
        "metric": "chi0*dV applications/s (mixed precision + FP64 refinement; eps err vs FP64 <= 1e-6)",
        "value": round(value, 3),
        "unit": "applications/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3+f32+f64" if main_mode == "bf16x3" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.L[0]:g}x{w.L[1]:g}x{w.L[2]:g} bohr, grid "
                               f"{w.n[0]}x{w.n[1]}x{w.n[2]}, ecut {w.ecut:g} Ha, N_pw {ctx.n_pw}, "
                               f"{w.n_wells} wells, N_v {w.n_v}, N_pdep {w.n_pdep}, seed {w.seed}",
                   "rhs_per_step": w.n_v * w.n_pdep, "cg_tol": w.cg_tol, "precision": main_mode},
        "eps_err_vs_fp64": eps_err,
        "eps_err_ok": (eps_err is not None and eps_err <= 1e-6),
        "fp64": fp64,
        "other_mixed_mode": other,
        "cg_iter_max": stats[-1]["cg_iter_max"],
        "cg_iter_mean": round(stats[-1]["cg_iter_total"] / max(stats[-1]["n_rhs"], 1), 2),
        "refine_steps": stats[-1]["refine_steps"],
        "fft_chunk_rows": stats[-1]["fft_chunk"],
        "setup_s": round(setup_s, 2),
        "dominant_kernel": kname,
        "roofline": roof,
        "kernels_one_step": {k: {"ms": round(v["ms"], 2), "launches": v["launches"]} for k, v in prof.items()
                             if v["launches"]},
        "pdep_eigs": eigs,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
