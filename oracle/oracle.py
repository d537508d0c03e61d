"""TEST INFRASTRUCTURE -- NOT PART OF THE PRODUCT PATH.

ctypes binding of the plain FP64 CPU oracle (``oracle/kbe_oracle.cpp``) of the
Kadanoff-Baym propagation step of arXiv 2505.19467. Only the tests, the smoke
check and the benchmark's CPU-baseline leg import this module.

Array conventions (oracle-private, numpy complex128):
  row j of the two-time lower triangle ... (j+1, nk, 2, nb, nb) = [t'][k][</>][a][b]
  Sigma row / collision row ............... (m+1, nk, 2, nb, nb) = [t_j or t'][k][</>][a][b]
  density matrix .......................... (nk, nb, nb)
  observables ............................. (nt+1, NOBS), columns named in OBS_NAMES
k is flattened as k = ix * nky + iy, with k_j = -pi + 2 pi j / n per axis (eq. (kj)).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kbe_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

OBS_NAMES = ["t", "N", "Ekin", "EHF", "Ecorr", "Etot", "Jx", "Jy", "A",
             "n_orb0", "n_orb1", "n_orb2", "n_orb3",
             "n_band0", "n_band1", "n_band2", "n_band3"]
NOBS = len(OBS_NAMES)
OBS = {n: i for i, n in enumerate(OBS_NAMES)}


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (plain -O2, OpenMP over k-points)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        # link to a private file and rename it into place, so that a process that has the
        # library loaded (a long reference run) keeps its own copy
        tmp = f"{_LIB}.{os.getpid()}.tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class OracleParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("nkx", "nky", "nb", "spin_deg", "interaction", "hf", "corr", "n_corr", "nt", "quad_points",
                 "pulse_kind")] + \
               [(n, ctypes.c_double) for n in
                ("dt", "U", "temp", "filling", "amp", "omega", "t0", "width", "polx", "poly", "corr_tol")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        P = ctypes.POINTER(OracleParams)
        _lib.oracle_run.argtypes = [P, dp, ctypes.c_int32, dp, dp, dp, dp]
        _lib.oracle_sigma_row.argtypes = [P, ctypes.c_int32, dp, dp]
        _lib.oracle_collision_row.argtypes = [P, ctypes.c_int32, dp, dp, dp]
        _lib.oracle_propagators.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, dp, dp]
        _lib.oracle_eigh.argtypes = [ctypes.c_int32, ctypes.c_int32, dp, dp, dp]
        _lib.oracle_initial_state.argtypes = [P, dp, dp, dp]
        _lib.oracle_h0.argtypes = [P, dp, ctypes.c_double, dp]
        _lib.oracle_tlm_run.argtypes = [P, dp, ctypes.c_int32, dp, dp]
        ip = ctypes.POINTER(ctypes.c_int32)
        _lib.oracle_run_log.argtypes = [P, dp, ctypes.c_int32, dp, ip, dp, ip]
        _lib.oracle_quad_weights.argtypes = [ctypes.c_int32, ctypes.c_int32, dp]
        _lib.oracle_full_square_check.argtypes = [P, dp, ctypes.c_int32, dp]
        _lib.oracle_max_threads.restype = ctypes.c_int
        _lib.oracle_set_threads.argtypes = [ctypes.c_int32]
        _lib.oracle_set_progress.argtypes = [ctypes.c_int32]
    return _lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"] and a.dtype in (np.float64, np.complex128)
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def params(cfg) -> OracleParams:
    pu = cfg.pulse
    return OracleParams(nkx=cfg.nkx, nky=cfg.nky, nb=cfg.nb, spin_deg=cfg.spin_deg,
                        interaction=cfg.interaction, hf=cfg.hf, corr=cfg.corr, n_corr=cfg.n_corr,
                        nt=cfg.nt, quad_points=cfg.quad_points, pulse_kind=pu.kind, dt=cfg.dt, U=cfg.U, temp=cfg.temp, filling=cfg.filling,
                        amp=pu.amp, omega=pu.omega, t0=pu.t0, width=pu.width,
                        polx=pu.pol[0], poly=pu.pol[1], corr_tol=cfg.corr_tol)


def _hop(cfg) -> np.ndarray:
    return np.ascontiguousarray(cfg.hop, dtype=np.complex128)


def run(cfg, nsteps: int | None = None, history: bool = False):
    """Propagate ``nsteps`` (default cfg.nt) steps. Returns dict with 'obs',
    'final_row', 'rho' and, if requested, 'rows' (list of row arrays)."""
    n = cfg.nt if nsteps is None else nsteps
    nk, nb = cfg.nk, cfg.nb
    blk = 2 * nb * nb
    obs = np.zeros((n + 1, NOBS))
    final = np.zeros((n + 1, nk, 2, nb, nb), np.complex128)
    rho = np.zeros((nk, nb, nb), np.complex128)
    hist = None
    if history:
        tot = sum((j + 1) for j in range(n + 1)) * nk * blk
        hist = np.zeros(tot, np.complex128)
    p = params(cfg)
    rc = lib().oracle_run(ctypes.byref(p), _ptr(_hop(cfg)), n, _ptr(obs), _ptr(final), _ptr(hist), _ptr(rho))
    if rc != 0:
        raise ValueError(f"oracle_run rejected the configuration (rc={rc})")
    out = {"obs": obs, "final_row": final, "rho": rho}
    if history:
        rows, off = [], 0
        for j in range(n + 1):
            sz = (j + 1) * nk * blk
            rows.append(hist[off:off + sz].reshape(j + 1, nk, 2, nb, nb))
            off += sz
        out["rows"] = rows
    return out


def quad_weights(quad_points: int, N: int) -> np.ndarray:
    """Weights of the collision-integral quadrature on the nodes 0..N (trapezoid for
    quad_points = 1, Gregory end corrections with quad_points nodes per end otherwise)."""
    out = np.zeros(N + 1)
    rc = lib().oracle_quad_weights(quad_points, N, _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_quad_weights rejected quad_points={quad_points}, N={N}")
    return out


def run_log(cfg, nsteps: int | None = None, with_unconverged: bool = False):
    """Propagation with the corrector log (Algorithm "prop"'s max / epsilon loop).
    Returns (obs, passes, changes): passes[m] corrector passes of step m, changes[m - 1, i] the
    row change after pass i of step m (-1: no such pass; only with cfg.corr_tol > 0); with
    ``with_unconverged`` also unconverged[m] = 1 where step m ran all n_corr passes with its
    last change still above cfg.corr_tol."""
    n = cfg.nt if nsteps is None else nsteps
    obs = np.zeros((n + 1, NOBS))
    passes = np.zeros(n + 1, np.int32)
    unconv = np.zeros(n + 1, np.int32)
    changes = np.zeros((max(n, 1), max(cfg.n_corr, 1)))
    p = params(cfg)
    ip = ctypes.POINTER(ctypes.c_int32)
    rc = lib().oracle_run_log(ctypes.byref(p), _ptr(_hop(cfg)), n, _ptr(obs), passes.ctypes.data_as(ip),
                              _ptr(changes), unconv.ctypes.data_as(ip))
    if rc != 0:
        raise ValueError(f"oracle_run_log rejected the configuration (rc={rc})")
    if with_unconverged:
        return obs, passes, changes[:n, :cfg.n_corr], unconv
    return obs, passes, changes[:n, :cfg.n_corr]


def tlm_run(cfg, nsteps: int | None = None):
    """Tangent-linear run (forward-mode dual numbers through the whole propagation).
    Returns (obs, dobs) with dobs[m, i, q] = d obs[m, i] / d(amp, omega, U)[q]."""
    n = cfg.nt if nsteps is None else nsteps
    obs = np.zeros((n + 1, NOBS))
    dobs = np.zeros((n + 1, NOBS, 3))
    p = params(cfg)
    rc = lib().oracle_tlm_run(ctypes.byref(p), _ptr(_hop(cfg)), n, _ptr(obs), _ptr(dobs))
    if rc != 0:
        raise ValueError(f"oracle_tlm_run rejected the configuration (rc={rc})")
    return obs, dobs


def full_square_check(cfg, nsteps: int):
    """Full-square propagation (upper triangle from the t'-equation with right-form collision
    integrals). Returns (asymmetry max|G(t,t') + G(t',t)^dag| / max|G|, max|rho - rho^dag|,
    max relative difference of the lower triangle from the plain run)."""
    out = np.zeros(3)
    p = params(cfg)
    rc = lib().oracle_full_square_check(ctypes.byref(p), _ptr(_hop(cfg)), nsteps, _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_full_square_check rejected the configuration (rc={rc})")
    return tuple(out)


def sigma_row(cfg, m: int, row: np.ndarray) -> np.ndarray:
    row = np.ascontiguousarray(row, np.complex128)
    assert row.shape == (m + 1, cfg.nk, 2, cfg.nb, cfg.nb)
    out = np.zeros_like(row)
    p = params(cfg)
    lib().oracle_sigma_row(ctypes.byref(p), m, _ptr(row), _ptr(out))
    return out


def collision_row(cfg, m: int, rows, sig: np.ndarray) -> np.ndarray:
    """I(t_m, t') for t' = 0..m from history rows 0..m and the Sigma row of t_m."""
    hist = np.ascontiguousarray(np.concatenate([np.asarray(r, np.complex128).ravel() for r in rows[:m + 1]]))
    sig = np.ascontiguousarray(sig, np.complex128)
    assert sig.shape == (m + 1, cfg.nk, 2, cfg.nb, cfg.nb)
    out = np.zeros_like(sig)
    p = params(cfg)
    lib().oracle_collision_row(ctypes.byref(p), m, _ptr(hist), _ptr(sig), _ptr(out))
    return out


def propagators(hbar: np.ndarray, dt: float) -> np.ndarray:
    """V, Vh, Phi for each Hermitian matrix in hbar (count, nb, nb) -> (count, 3, nb, nb)."""
    hbar = np.ascontiguousarray(hbar, np.complex128)
    cnt, nb, _ = hbar.shape
    out = np.zeros((cnt, 3, nb, nb), np.complex128)
    lib().oracle_propagators(nb, cnt, dt, _ptr(hbar), _ptr(out))
    return out


def eigh(A: np.ndarray):
    A = np.ascontiguousarray(A, np.complex128)
    cnt, nb, _ = A.shape
    w = np.zeros((cnt, nb))
    v = np.zeros_like(A)
    lib().oracle_eigh(nb, cnt, _ptr(A), _ptr(w), _ptr(v))
    return w, v


def initial_state(cfg):
    rho = np.zeros((cfg.nk, cfg.nb, cfg.nb), np.complex128)
    mu = ctypes.c_double(0.0)
    p = params(cfg)
    lib().oracle_initial_state(ctypes.byref(p), _ptr(_hop(cfg)), _ptr(rho), ctypes.byref(mu))
    return rho, mu.value


def h0(cfg, A: float) -> np.ndarray:
    out = np.zeros((cfg.nk, cfg.nb, cfg.nb), np.complex128)
    p = params(cfg)
    lib().oracle_h0(ctypes.byref(p), _ptr(_hop(cfg)), float(A), _ptr(out))
    return out


def max_threads() -> int:
    """Threads the oracle's OpenMP loops over k-points use."""
    return int(lib().oracle_max_threads())


def set_threads(n: int) -> None:
    """Set the oracle's OpenMP thread count (for a one-core timing)."""
    lib().oracle_set_threads(int(n))


def set_progress(every: int) -> None:
    """every > 0: the runs print "[oracle] step m of n" to stderr after every ``every`` steps
    (long timing runs); 0 turns it off."""
    lib().oracle_set_progress(int(every))
