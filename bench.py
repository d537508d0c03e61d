"""Benchmark: KBE propagation steps/s and history-sum HBM bandwidth on one MI355X.

Workload: the 2D square-lattice system with a 24x24 k-grid, nb = 2 orbitals, seeded
+-10% hoppings/on-site energies/U, Gaussian-envelope pulse along x, dt = 0.02,
nt = 1000 steps, FP64 (complex128), one corrector pass per step (two history passes).
Synthetic, seeded input; no dataset.

A "step" is one KBE time step: self-energy slice, history sums, end points and the
predictor-corrector update of G(t_m, .) and rho_m, and the observables.

Prints one JSON line. Every run propagates the whole trajectory (nt steps from t = 0).
``--steps K`` times its LAST K steps, nt - K + 1 .. nt, which run against the full-length
history (steps 1 .. nt - K run first, untimed for ``value``); the default K = nt times the
whole trajectory. The whole trajectory's steps/s and history-sum bandwidth are reported
beside the timed window in every case. ``--warmup W`` steps are run first on the same
buffers and then discarded (the context is re-created at t = 0 before the trajectory).
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

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E

# HBM traffic of the FP64 history-sum kernel per launch: rocprofv3 FETCH_SIZE and WRITE_SIZE runs,
# scaled by what the same counters read for a plain 1 GiB device copy (x2.000 and x1.000), averaged
# over the launches of the timed window (the last K steps of the trajectory), keyed by (workload,
# nt, timed steps K); summary and commands in profiles/k_hist_pair_c2_sq24_nb2.md. Valid only for
# the code it was measured on (SHA-1 of the k_hist_pair template and kbe_device.hpp, comments
# removed); reported as null once that code changes, or for a window that was not measured.
MEASURED_TRAFFIC = {"bytes_per_launch": {("c2", 1000, 20): 3.70684e10, ("c2", 1000, 1000): 1.26860e10},
                    "source_sha1": "7def1ccecd3e767c4a0d16a42dea89f26572e628"}


def _kernel_source_sha1():
    """SHA-1 of the FP64 history-sum kernel's code (the k_hist_pair template) and of the shared
    device header, comments and blank lines removed: code changes of that kernel only."""
    import hashlib
    import re
    d = os.path.join(ROOT, "paper_2505_19467_amd", "csrc")

    def code(text):
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        return [ln.split("//")[0].rstrip() for ln in text.splitlines()]
    k = open(os.path.join(d, "kbe_kernels.hip")).read()
    a = k.index("__global__ __launch_bounds__(256) void k_hist_pair(")
    b = k.index("// ------------------------------------------------------------------", a)
    lines = code(k[a:b]) + code(open(os.path.join(d, "kbe_device.hpp")).read())
    return hashlib.sha1("\n".join(ln for ln in lines if ln).encode()).hexdigest()


def _rel_devs(obs, ref, names):
    """Largest deviation of each observable series from a reference run, relative to the
    series' largest magnitude; series that vanish by symmetry (|ref| < 1e-12) are left out."""
    out = {}
    for n, i in names.items():
        scale = np.abs(ref[:, i]).max()
        if scale >= 1e-12:
            out[n] = float(np.abs(obs[:, i] - ref[:, i]).max() / scale)
    return out


def _energy_balance(obs, cfg):
    """E_tot(t) - E_tot(0) + int A'(t) J(t) dt for the Peierls pulse (None for the dipole kick,
    which injects energy at one instant)."""
    pu = cfg.pulse
    if getattr(pu, "kind", 0) != 0:
        return None
    t = obs[:, 0]
    g = np.exp(-((t - pu.t0) / pu.width) ** 2)
    Adot = pu.amp * (pu.omega * np.cos(pu.omega * t) * g - np.sin(pu.omega * t) * g * 2 * (t - pu.t0) / pu.width ** 2)
    J = obs[:, 6] * pu.pol[0] + obs[:, 7] * pu.pol[1]
    f = Adot * J
    W = np.concatenate([[0.0], np.cumsum(0.5 * (f[1:] + f[:-1]) * cfg.dt)])
    return obs[:, 5] - obs[0, 5] + W


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, sample_steps: int, same_steps: int):
    """The CPU oracle (plain FP64 C++, OpenMP over k) on the first ``sample_steps`` steps of the
    same workload with all its threads; then the first ``same_steps`` steps with all threads and
    with one thread (one sample for both rates)."""
    from oracle import oracle as O
    O.build()
    threads = O.max_threads()
    t0 = time.perf_counter()
    O.run(cfg, sample_steps)
    dt = time.perf_counter() - t0
    dt_same = dt1 = None
    if same_steps > 0:
        t0 = time.perf_counter()
        O.run(cfg, same_steps)
        dt_same = time.perf_counter() - t0
        O.set_threads(1)
        t0 = time.perf_counter()
        O.run(cfg, same_steps)
        dt1 = time.perf_counter() - t0
        O.set_threads(threads)
    return dt, threads, dt_same, dt1


def cpu_extended(what: str):
    """Longer CPU-oracle baselines beside the GPU path on the same workload, one per call
    (each is minutes of oracle work on the host's cores, so none runs by default):

    * ``c1``: the 16-point chain, nb = 2, all 200 steps: oracle with all threads and with one;
    * ``c4``: the 12x12 gradient workload, all 400 steps: oracle forward run; an FD gradient of
      its three parameters by central differences costs six such runs; GPU forward run and
      reverse sweep;
    * ``c4_tlm``: the oracle's tangent-linear run of the same 400 steps (the CPU way to the
      gradient that the reverse sweep computes);
    * ``c5_400``: the 16x16, nb = 4 workload truncated to n_t = 400, oracle and GPU.

    The oracle prints a progress line every 5 % of the steps."""
    import torch
    from oracle import oracle as O
    from paper_2505_19467_amd import inputs, kbe
    O.build()
    threads = O.max_threads()
    if what == "c1":
        cfg = inputs.c1()
    elif what in ("c4", "c4_tlm"):
        cfg = inputs.c4()
    elif what == "c5_400":
        cfg = inputs.c5().replace(nt=400)
    else:
        raise SystemExit(f"bench.py: unknown --cpu-extended workload {what!r} (c1, c4, c4_tlm, c5_400)")
    n = cfg.nt
    O.set_progress(max(1, n // 20))

    def oracle_time(fn, nthreads=None):
        if nthreads:
            O.set_threads(nthreads)
        t0 = time.perf_counter()
        fn()
        el = time.perf_counter() - t0
        O.set_threads(threads)
        print(f"[bench] oracle {what}: {el:.1f} s with {nthreads or threads} threads", file=sys.stderr, flush=True)
        return el

    out = {"workload": cfg.name, "steps": n, "cpu_model": cpu_model(), "threads": threads, "kind": "oracle"}
    if what == "c4_tlm":
        out["tlm_s"] = oracle_time(lambda: O.tlm_run(cfg, n))
        print(json.dumps(out), flush=True)
        return
    out["oracle_s"] = oracle_time(lambda: O.run(cfg, n))
    if what == "c1":
        out["oracle_one_thread_s"] = oracle_time(lambda: O.run(cfg, n), 1)
    if what == "c4":
        out["fd_gradient_s_derived"] = 6 * out["oracle_s"]
    S = kbe.System(cfg)
    S.step(min(5, n))
    S.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.step(n)
    torch.cuda.synchronize()
    out["gpu_s"] = time.perf_counter() - t0
    if what == "c4":
        t0 = time.perf_counter()
        S.adjoint_gradient("n_band1")
        torch.cuda.synchronize()
        out["gpu_reverse_s"] = time.perf_counter() - t0
    S.close()
    out["oracle_steps_per_s"] = n / out["oracle_s"]
    out["gpu_steps_per_s"] = n / out["gpu_s"]
    print(f"[bench] {what}: oracle {out['oracle_s']:.1f} s, GPU {out['gpu_s']:.3f} s", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


def adjoint_leg(torch, inputs, kbe):
    """Gradient workload: the 12x12-k, nb = 2, 400-step system; forward propagation (its
    history is the reverse sweep's checkpoint store), then the reverse sweep for
    d n_band1(T) / d(amp, omega, U)."""
    cfg = inputs.c4()
    n = cfg.nt
    S = kbe.System(cfg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.step(n)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    t0 = time.perf_counter()
    g = S.adjoint_gradient("n_band1")
    torch.cuda.synchronize()
    tr = time.perf_counter() - t0
    S.close()
    print(f"[bench] adjoint ({cfg.name}, {n} steps): forward {tf:.3f} s, reverse {tr:.3f} s, "
          f"grad {g}", file=sys.stderr, flush=True)
    return {"workload": f"{cfg.name}: 2D 12x12 k-grid, nb=2, nt={n}, dt={cfg.dt}, loss n_band1(T)",
            "forward_s": tf, "reverse_s": tr, "reverse_over_forward": tr / tf,
            "grad_amp_omega_U": [float(x) for x in g]}


def paper_leg(torch, inputs, kbe, warmup: int, reps: int = 5):
    """The paper's own workload (two-band chain, n_k = 1024, interband U, dipole kick, FP64):
    steps 1..499 timed as a whole, then the step at n_t = 500 run stage by stage with its
    self-energy slice and its collision integrals (history sums, end points, equal-time term)
    timed on their own, as the paper reports its two components."""
    cfg = inputs.paper_chain()
    S = kbe.System(cfg)
    if warmup:
        S.step(min(warmup, cfg.nt - 1))
        S.observables()
    S.reset()
    n = cfg.nt - 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.step(n)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    m = cfg.nt
    S.stage_propagators(m, 0)
    S.stage_update(m, 0)
    torch.cuda.synchronize()

    def timed(fn, n_rep=reps):
        best = []
        for _ in range(n_rep):
            a = time.perf_counter()
            fn(m)
            torch.cuda.synchronize()
            best.append(time.perf_counter() - a)
        return 1e3 * float(np.median(best))
    sig_ms = timed(S.stage_sigma)
    ci_ms = timed(S.stage_collision)
    # the paper's own self-energy algorithm (direct momentum sums) on the same slice
    dir_ms = timed(S.stage_sigma_direct, 2)
    obs = S.observables(0, n + 1)
    S.close()
    out = {"value": n / el, "unit": "steps/s", "steps": n,
           "sigma_ms_at_nt500": sig_ms, "collision_ms_at_nt500": ci_ms,
           "sigma_direct_sums_ms_at_nt500": dir_ms,
           "n_band1_final": float(obs[-1, 14]), "N_drift": float(np.abs(obs[:, 1] - obs[0, 1]).max()),
           "paper_16_A100_s": {"sigma_cuda_fortran": 9.06, "collision_openacc": 7.83},
           "workload": f"{cfg.name}: 1D two-band chain, n_k={cfg.nk}, interband U={cfg.U}, dipole kick "
                       f"I={cfg.pulse.amp} at t={cfg.pulse.t0}, dt={cfg.dt}, K={cfg.n_corr}, FP64"}
    print(f"[bench] paper workload: {n} steps in {el:.3f} s = {n / el:.1f} steps/s; at n_t = 500 the "
          f"self-energy slice takes {sig_ms:.3f} ms ({dir_ms:.1f} ms by the paper's direct sums) and the "
          f"collision integrals {ci_ms:.3f} ms",
          file=sys.stderr, flush=True)
    return out


def hbm_ceiling(torch, gib: float = 4.0, reps: int = 5):
    """Plain device-to-device copy (read + write) and a full-array sum (read) with torch's
    own kernels, as a measured ceiling beside the 8 TB/s peak."""
    n = int(gib * 2 ** 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    a.sum()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * n * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    e0.record()
    for _ in range(reps):
        a.sum()
    e1.record()
    torch.cuda.synchronize()
    read_gbs = n * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    print(f"[bench] HBM probe: copy {copy_gbs:.0f} GB/s (read + write), sum {read_gbs:.0f} GB/s (read)",
          file=sys.stderr, flush=True)
    return {"copy_GBs": copy_gbs, "read_GBs": read_gbs, "bytes_each": n * 8}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--cpu-sample", type=int, default=120, help="oracle steps for the CPU baseline (0: skip)")
    ap.add_argument("--cpu-sample-one-core", type=int, default=40,
                    help="oracle steps timed with all threads and with one (the core-scaling sample)")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-form run")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint (gradient) leg")
    ap.add_argument("--no-adaptive", action="store_true",
                    help="skip the run with the corrector's stopping rule (tolerance mode)")
    ap.add_argument("--no-gregory", action="store_true",
                    help="skip the run with Gregory end corrections of the collision-integral quadrature")
    ap.add_argument("--no-paper", action="store_true",
                    help="skip the paper's own workload (two-band chain, n_k = 1024, 500 steps, per-phase times)")
    ap.add_argument("--no-ceiling", action="store_true", help="skip the plain copy/read bandwidth probe")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="do not record HIP events around the history-sum launches (for counter-collection runs)")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="only run one device-to-device copy of GIB GiB (to scale HBM byte counters) and exit")
    ap.add_argument("--cpu-extended", default=None, metavar="WORKLOAD",
                    help="only time the CPU oracle on a longer workload beside the GPU (c1, c4, c4_tlm, "
                         "c5_400) and exit")
    args = ap.parse_args()
    if args.cpu_extended:
        cpu_extended(args.cpu_extended)
        return
    if args.copy_calibration > 0:
        import torch
        n = int(args.copy_calibration * 2 ** 30) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": n * 8}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this library runs on one GPU only (asked for --gpus {args.gpus}); "
              "the k-point sharding across GPUs is described in the design notes, not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2505_19467_amd import inputs, kbe

    cfg = inputs.WORKLOADS[args.workload]()
    K = cfg.nt if args.steps is None else args.steps
    W = args.warmup
    if K < 1 or K > cfg.nt or W < 0 or W > cfg.nt:
        print(f"bench.py: --steps must be in 1..{cfg.nt} and --warmup in 0..{cfg.nt}", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    print(f"[bench] workload {cfg.name}: nk={cfg.nk} nb={cfg.nb} nt={cfg.nt} dt={cfg.dt} K={cfg.n_corr}; "
          f"timing {K} steps after {W} warm-up steps", file=sys.stderr, flush=True)

    kt = not args.no_kernel_timing

    def run(c):
        """The whole trajectory of ``c``; steps nt - K + 1 .. nt are the timed window."""
        S = kbe.System(c)
        gb = S.history.numel() * S.history.element_size() / 1e9
        if W:
            S.step(W)
            S.observables()
        S.reset()   # fresh context on the same buffers: t = 0 again
        pre = c.nt - K
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if pre:
            S.timing(kt)
            S.step(pre)
            torch.cuda.synchronize()
        t_pre = time.perf_counter() - t0
        pl, pms, pbytes = S.timing_query() if (pre and kt) else (0, 0.0, 0.0)
        S.timing(kt)   # the window's history-sum launches only
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.step(K)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        launches, kms, kbytes = S.timing_query()
        obs = S.observables(0, c.nt + 1)
        whole = t_pre + el
        wl, wms, wbytes = launches + pl, kms + pms, kbytes + pbytes
        traj = {"steps": c.nt, "steps_per_s": c.nt / whole,
                "history_sums_GBs": wbytes / (wms * 1e-3) / 1e9 if wms > 0 else None,
                "history_sums_launches": wl}
        return S, dict(elapsed=el, launches=launches, kms=kms, kbytes=kbytes, obs=obs, hist_gb=gb,
                       whole_s=whole, traj=traj)

    S, r64 = run(cfg)
    elapsed, obs, hist_gb = r64["elapsed"], r64["obs"], r64["hist_gb"]
    launches, kms, kbytes = r64["launches"], r64["kms"], r64["kbytes"]
    steps_per_s = K / elapsed
    achieved = kbytes / (kms * 1e-3) / 1e9 if kms > 0 else None
    n_drift = float(np.abs(obs[:, 1] - obs[0, 1]).max())
    eb = _energy_balance(obs, cfg)
    e_bal = float(np.abs(eb).max()) if eb is not None else None
    finite = bool(np.isfinite(obs).all())
    first = cfg.nt - K + 1
    traj = r64["traj"]
    print(f"[bench] FP64: steps {first}..{cfg.nt} in {elapsed:.3f} s = {steps_per_s:.1f} steps/s; history sums: "
          f"{launches} launches, {kms:.1f} ms, {kbytes / 1e12:.3f} TB algorithmic -> {achieved or 0:.0f} GB/s; "
          f"whole trajectory {traj['steps_per_s']:.1f} steps/s, {traj['history_sums_GBs'] or 0:.0f} GB/s; "
          f"N drift {n_drift:.1e}, energy balance " + (f"{e_bal:.1e}" if e_bal is not None else "n/a (dipole kick)"),
          file=sys.stderr, flush=True)

    def fresh(S):
        S.close()
        del S
        torch.cuda.empty_cache()

    fp32 = None
    if not args.no_fp32:
        fresh(S)
        c32 = cfg.replace(precision=inputs.PRECISION_FP32)
        S, r32 = run(c32)
        o32 = r32["obs"]
        names = {"n_band1": 14, "n_band0": 13, "n_orb0": 9, "n_orb1": 10, "Jx": 6, "Etot": 5, "N": 1}
        err = _rel_devs(o32, obs, names)
        ach32 = r32["kbytes"] / (r32["kms"] * 1e-3) / 1e9 if r32["kms"] > 0 else None
        fp32 = {"value": K / r32["elapsed"], "unit": "steps/s", "speedup_vs_fp64": elapsed / r32["elapsed"],
                "history_sums_GBs": ach32, "history_sums_frac": ach32 / HBM_PEAK_GBS if ach32 else None,
                "trajectory": r32["traj"], "trajectory_speedup_vs_fp64": r64["whole_s"] / r32["whole_s"],
                "history_GB": round(r32["hist_gb"], 2),
                "max_rel_err_vs_fp64": err, "error_over_steps": f"0..{cfg.nt}", "kernel": "k_hist_pair32"
                if cfg.nb <= 2 else ("k_hist_bulk32_split" if cfg.nb == 4 else "k_hist_bulk32"),
                "workload": f"{c32.name}: history stored and summed in FP32 on the vector ALU"}
        print(f"[bench] FP32 form: steps {first}..{cfg.nt} in {r32['elapsed']:.3f} s = {K / r32['elapsed']:.1f} "
              f"steps/s ({elapsed / r32['elapsed']:.2f}x); history sums {ach32 or 0:.0f} GB/s; whole trajectory "
              f"{r32['traj']['steps_per_s']:.1f} steps/s ({r64['whole_s'] / r32['whole_s']:.2f}x); max rel err vs "
              f"FP64 over {cfg.nt} steps {max(err.values()):.1e}", file=sys.stderr, flush=True)
        fresh(S)
        S = kbe.System(cfg)

    mfma = None
    if not args.no_fp32:
        fresh(S)
        cm = cfg.replace(precision=inputs.PRECISION_FP32_MFMA)
        S, rm = run(cm)
        names = {"n_band1": 14, "n_band0": 13, "n_orb0": 9, "n_orb1": 10, "Jx": 6, "Etot": 5, "N": 1}
        err = _rel_devs(rm["obs"], obs, names)
        achm = rm["kbytes"] / (rm["kms"] * 1e-3) / 1e9 if rm["kms"] > 0 else None
        mfma = {"value": K / rm["elapsed"], "unit": "steps/s", "speedup_vs_fp64": elapsed / rm["elapsed"],
                "history_sums_GBs": achm, "history_sums_frac": achm / HBM_PEAK_GBS if achm else None,
                "kernel": "k_hist_mfma",
                "trajectory": rm["traj"], "trajectory_speedup_vs_fp64": r64["whole_s"] / rm["whole_s"],
                "history_GB": round(rm["hist_gb"], 2),
                "max_rel_err_vs_fp64": err, "error_over_steps": f"0..{cfg.nt}",
                "workload": f"{cm.name}: FP32 history, column sums on FP32 MFMA with hi/lo split Sigma"}
        print(f"[bench] FP32-MFMA form: steps {first}..{cfg.nt} in {rm['elapsed']:.3f} s = {K / rm['elapsed']:.1f} "
              f"steps/s ({elapsed / rm['elapsed']:.2f}x); history sums {achm or 0:.0f} GB/s; whole trajectory "
              f"{rm['traj']['steps_per_s']:.1f} steps/s ({r64['whole_s'] / rm['whole_s']:.2f}x); max rel err vs "
              f"FP64 over {cfg.nt} steps {max(err.values()):.1e}", file=sys.stderr, flush=True)
        fresh(S)
        S = kbe.System(cfg)

    adaptive = None
    if not args.no_adaptive and args.workload == "c2":
        # Algorithm "prop"'s stopping rule on the same workload: at most 4 corrector passes, stop
        # once the row changes by <= 6e-9 (a wide gap of the changes: 3 passes on every step)
        fresh(S)
        ca = cfg.replace(n_corr=4, corr_tol=6e-9)
        S, ra = run(ca)
        passes, _ = S.corrector_log(1, cfg.nt)
        oa = ra["obs"]
        dev = _rel_devs(oa, obs, {"n_band1": 14, "Jx": 6, "Etot": 5})
        adaptive = {"value": K / ra["elapsed"], "unit": "steps/s", "trajectory": ra["traj"],
                    "corr_tol": ca.corr_tol, "max_passes": ca.n_corr,
                    "mean_passes": float(passes.mean()), "pass_histogram": np.bincount(passes).tolist(),
                    "history_passes_per_step": 1.0 + float(passes.mean()),
                    "max_rel_dev_vs_one_pass": dev,
                    "workload": f"{ca.name}: corrector passes until the row changes by <= {ca.corr_tol:g} "
                                f"(at most {ca.n_corr}), FP64"}
        print(f"[bench] stopping rule: steps {first}..{cfg.nt} in {ra['elapsed']:.3f} s = {K / ra['elapsed']:.1f} "
              f"steps/s; {passes.mean():.2f} corrector passes per step; deviation from one pass "
              f"{max(dev.values()):.1e}", file=sys.stderr, flush=True)
        fresh(S)
        S = kbe.System(cfg)

    gregory = None
    if not args.no_gregory and args.workload == "c2":
        # the same workload with the quadrature's higher-order end corrections (5 nodes per end)
        fresh(S)
        cq = cfg.replace(quad_points=5)
        S, rq = run(cq)
        oq = rq["obs"]
        dev = _rel_devs(oq, obs, {"n_band1": 14, "Jx": 6, "Etot": 5, "Ecorr": 3})
        achq = rq["kbytes"] / (rq["kms"] * 1e-3) / 1e9 if rq["kms"] > 0 else None
        gregory = {"value": K / rq["elapsed"], "unit": "steps/s", "trajectory": rq["traj"],
                   "quad_points": cq.quad_points,
                   "history_sums_GBs": achq, "max_rel_dev_vs_trapezoid": dev,
                   "N_drift": float(np.abs(oq[:, 1] - oq[0, 1]).max()),
                   "energy_balance_max": float(np.abs(_energy_balance(oq, cq)).max()),  # Peierls pulse
                   "workload": f"{cq.name}: Gregory end corrections, {cq.quad_points} nodes per end, FP64"}
        print(f"[bench] Gregory q={cq.quad_points}: steps {first}..{cfg.nt} in {rq['elapsed']:.3f} s = "
              f"{K / rq['elapsed']:.1f} steps/s; deviation from the trapezoid {max(dev.values()):.1e}",
              file=sys.stderr, flush=True)
        fresh(S)
        S = kbe.System(cfg)

    paper = None
    if not args.no_paper and args.workload == "c2":
        fresh(S)
        paper = paper_leg(torch, inputs, kbe, W)
        S = kbe.System(cfg)

    adj = None
    if not args.no_adjoint:
        fresh(S)
        adj = adjoint_leg(torch, inputs, kbe)
        S = kbe.System(cfg)

    ceiling = None
    if not args.no_ceiling:
        ceiling = hbm_ceiling(torch)

    cpu = None
    if args.cpu_sample > 0:
        ns = min(args.cpu_sample, cfg.nt)
        n1 = min(args.cpu_sample_one_core, ns)
        print(f"[bench] CPU oracle on steps 1..{ns}, and on steps 1..{n1} with all threads and with one ...",
              file=sys.stderr, flush=True)
        tcpu, threads, tcpu_same, tcpu1 = cpu_baseline(cfg, ns, n1)
        # GPU time for the same steps, for a like-for-like ratio
        S.reset()
        torch.cuda.synchronize()
        tg0 = time.perf_counter()
        S.step(ns)
        torch.cuda.synchronize()
        tgpu = time.perf_counter() - tg0
        cpu = {"value": ns / tcpu, "unit": "steps/s", "cores": threads, "kind": "oracle",
               "sample": f"{cfg.name} steps 1..{ns} of {cfg.nt} (FP64 C++ oracle, OpenMP over k); "
                         f"{tcpu:.2f} s; the GPU path takes {tgpu:.3f} s on the same steps",
               "gpu_same_sample_steps_per_s": ns / tgpu, "cpu_model": cpu_model(),
               "same_sample_all_threads_steps_per_s": (n1 / tcpu_same) if tcpu_same else None,
               "one_core_steps_per_s": (n1 / tcpu1) if tcpu1 else None,
               "one_core_sample": f"steps 1..{n1}, timed with all {threads} threads and with one"}

    traffic = None
    if _kernel_source_sha1() == MEASURED_TRAFFIC["source_sha1"]:
        traffic = MEASURED_TRAFFIC["bytes_per_launch"].get((args.workload, cfg.nt, K))
    line = {
        "metric": "KBE steps/s (history sums: achieved HBM GB/s)",
        "value": steps_per_s,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * elapsed / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: 2D {cfg.nkx}x{cfg.nky} k-grid, nb={cfg.nb}, nt={cfg.nt}, dt={cfg.dt}, "
                               f"second Born + HF, K={cfg.n_corr} corrector pass, FP64",
                   "nk": cfg.nk, "nb": cfg.nb, "nt": cfg.nt, "timed_steps": [first, cfg.nt],
                   "history_rows_in_timed_steps": [first, cfg.nt + 1],
                   "history_passes_per_step": cfg.n_corr + 1, "history_GB": round(hist_gb, 2)},
        "trajectory": traj,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
                     "traffic_unit": "bytes per launch (HBM fetch + write)",
                     "kernel": "k_hist_pair" if cfg.nb <= 2 else ("k_hist_bulk_split" if cfg.nb == 4 else "k_hist_bulk"),
                     "launches": launches, "kernel_ms": kms,
                     "algorithmic_bytes_per_launch": kbytes / launches if launches else None},
        "cpu_baseline": cpu,
        "fp32_form": fp32,
        "fp32_mfma_form": mfma,
        "adaptive_corrector": adaptive,
        "gregory": gregory,
        "paper_workload": paper,
        "adjoint": adj,
        "hbm_ceiling": ceiling,
        "checks": {"N_drift": n_drift, "energy_balance_max": e_bal, "finite": finite},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
