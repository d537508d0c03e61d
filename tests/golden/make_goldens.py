"""Write the stored reference values of the long trajectories from the CPU oracle.

Calls nothing but ``oracle/`` (and the seeded parameter sets of ``inputs``, which hold no
arithmetic of the method). The GPU tests compare the HIP path's full runs with these files:

  c2_nt1000_obs.txt        the 24x24, nb = 2 workload propagated for all 1000 steps (Algorithm
                           "prop", K = 1, trapezoid): the observable series at every step
  c2_nt1000_final_row.txt  G^<,>(t_1000, t') of that run at three k-points and every 20th t'
                           (plus the last four)
  p1_nt100_obs.txt         the paper's own model on the chain of n_k = 1024 points (interband U,
                           dipole kick at t = 0.5, i.e. step 25), the first 100 steps: the
                           observable series at every step
  p1_nt100_final_row.txt   G^<,>(t_100, t') of that run at three k-points and every 10th t'
  c4_nt400_tlm.txt         the 12x12 gradient workload (400 steps, dt = 0.025): the final-time
                           upper-band occupation and its derivatives with respect to the pulse
                           amplitude, the pulse frequency and U from the oracle's tangent-linear
                           run (dual numbers through the same scheme), at every step

Usage: python tests/golden/make_goldens.py c2|p1|c4 [threads]
The 24x24 run holds its 37 GB history in host memory and takes a few hours on eight cores; the
chain's 100 steps take minutes (its O(n_k^2) line sums dominate).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2505_19467_amd import inputs  # noqa: E402

# observables stored per step (columns of the oracle's series)
OBS_COLS = ["t", "N", "Ekin", "EHF", "Ecorr", "Etot", "Jx", "Jy", "n_orb0", "n_orb1", "n_band0", "n_band1"]
# sampled final-row entries: k-points (k = ix * nky + iy) and columns t'
C2_K = (0, 301, 575)
P1_K = (0, 511, 1023)
P1_STEPS = 100


def c2_tprimes(nt: int):
    return sorted(set(range(0, nt + 1, 20)) | set(range(nt - 3, nt + 1)))


def p1_tprimes(n: int):
    return sorted(set(range(0, n + 1, 10)) | set(range(n - 3, n + 1)))


def _header(f, lines):
    for ln in lines:
        f.write(f"# {ln}\n")


def make_c2(threads: int | None):
    cfg = inputs.c2()
    if threads:
        O.set_threads(threads)
    t0 = time.perf_counter()
    out = O.run(cfg, cfg.nt)
    el = time.perf_counter() - t0
    obs, final = out["obs"], out["final_row"]
    cmd = f"python tests/golden/make_goldens.py c2 {threads or ''}".rstrip()
    with open(os.path.join(HERE, "c2_nt1000_obs.txt"), "w") as f:
        _header(f, [f"written by: {cmd}",
                    f"CPU oracle (FP64), workload {cfg.name}: 2D 24x24 k-grid, nb = 2, U = {cfg.U!r}, dt = {cfg.dt}, "
                    f"nt = {cfg.nt}, K = {cfg.n_corr}, trapezoid; Algorithm \"prop\", eq. (CI), eq. (2BSE)",
                    f"oracle time {el:.0f} s on {O.max_threads()} threads",
                    "columns: " + " ".join(OBS_COLS)])
        for m in range(cfg.nt + 1):
            f.write(" ".join(f"{obs[m, O.OBS[c]]:.17e}" for c in OBS_COLS) + "\n")
    with open(os.path.join(HERE, "c2_nt1000_final_row.txt"), "w") as f:
        _header(f, [f"written by: {cmd}",
                    f"G(t_{cfg.nt}, t') of the same run: columns k t' comp(0 lesser, 1 greater) a b re im"])
        for k in C2_K:
            for tp in c2_tprimes(cfg.nt):
                for c in range(2):
                    for a in range(cfg.nb):
                        for b in range(cfg.nb):
                            z = final[tp, k, c, a, b]
                            f.write(f"{k} {tp} {c} {a} {b} {z.real:.17e} {z.imag:.17e}\n")
    print(f"c2: {cfg.nt} steps in {el:.0f} s", flush=True)


def _write_run(cfg, n, obs, final, el, cmd, obs_name, row_name, ks, tprimes, what):
    with open(os.path.join(HERE, obs_name), "w") as f:
        _header(f, [f"written by: {cmd}", what,
                    f"oracle time {el:.0f} s on {O.max_threads()} threads",
                    "columns: " + " ".join(OBS_COLS)])
        for m in range(n + 1):
            f.write(" ".join(f"{obs[m, O.OBS[c]]:.17e}" for c in OBS_COLS) + "\n")
    with open(os.path.join(HERE, row_name), "w") as f:
        _header(f, [f"written by: {cmd}",
                    f"G(t_{n}, t') of the same run: columns k t' comp(0 lesser, 1 greater) a b re im"])
        for k in ks:
            for tp in tprimes:
                for c in range(2):
                    for a in range(cfg.nb):
                        for b in range(cfg.nb):
                            z = final[tp, k, c, a, b]
                            f.write(f"{k} {tp} {c} {a} {b} {z.real:.17e} {z.imag:.17e}\n")


def make_p1(threads: int | None):
    cfg = inputs.paper_chain()
    n = P1_STEPS
    if threads:
        O.set_threads(threads)
    t0 = time.perf_counter()
    out = O.run(cfg, n)
    el = time.perf_counter() - t0
    cmd = f"python tests/golden/make_goldens.py p1 {threads or ''}".rstrip()
    what = (f"CPU oracle (FP64), workload {cfg.name}: chain of n_k = {cfg.nk}, nb = 2, interband U = {cfg.U!r}, "
            f"dipole kick {cfg.pulse.amp!r} at t = {cfg.pulse.t0!r}, dt = {cfg.dt}, steps 0..{n} of nt = {cfg.nt}, "
            f"K = {cfg.n_corr}, trapezoid; Algorithm \"prop\", eq. (CI), eq. (2BSE), eq. (dipole)")
    _write_run(cfg, n, out["obs"], out["final_row"], el, cmd, "p1_nt100_obs.txt", "p1_nt100_final_row.txt",
               P1_K, p1_tprimes(n), what)
    print(f"p1: {n} steps in {el:.0f} s", flush=True)


def make_c4(threads: int | None):
    cfg = inputs.c4()
    if threads:
        O.set_threads(threads)
    t0 = time.perf_counter()
    obs, dobs = O.tlm_run(cfg, cfg.nt)
    el = time.perf_counter() - t0
    i = O.OBS["n_band1"]
    cmd = f"python tests/golden/make_goldens.py c4 {threads or ''}".rstrip()
    with open(os.path.join(HERE, "c4_nt400_tlm.txt"), "w") as f:
        _header(f, [f"written by: {cmd}",
                    f"CPU oracle tangent-linear run (dual numbers, FP64), workload {cfg.name}: 2D 12x12 k-grid, "
                    f"nb = 2, U = {cfg.U!r}, dt = {cfg.dt}, nt = {cfg.nt}, K = {cfg.n_corr}, trapezoid",
                    f"oracle time {el:.0f} s on {O.max_threads()} threads",
                    "columns: step n_band1 d/d_amp d/d_omega d/d_U"])
        for m in range(cfg.nt + 1):
            f.write(f"{m} {obs[m, i]:.17e} " + " ".join(f"{dobs[m, i, q]:.17e}" for q in range(3)) + "\n")
    print(f"c4: {cfg.nt} tangent-linear steps in {el:.0f} s", flush=True)


if __name__ == "__main__":
    which = sys.argv[1]
    thr = int(sys.argv[2]) if len(sys.argv) > 2 else None
    {"c2": make_c2, "p1": make_p1, "c4": make_c4}[which](thr)
