"""Independent numpy references used to pin the oracle (tests only).

Each function is written from a different formula than the oracle uses, so that a
plausible mistake in the oracle (a dropped term, a wrong sign, a transposed
operand, a wrong momentum index) shows up as a mismatch:

* ``paper_sigma_direct``: eq. (2BSE) as printed, the O(n_k^3) double momentum sum
  (direct minus exchange), with the momentum index map of Sec. "Trading on-the-fly
  index calculation" (``allind_kpk``) written from its three-case formula.
* ``hubbard_sigma_direct``: the spin-degenerate on-site Hubbard second-Born
  self-energy as a momentum-space convolution (double sum over k1, k2).
* ``tdhf_rk4``: time-dependent Hartree-Fock density matrix by classical RK4.
"""
from __future__ import annotations

import numpy as np


def kgrid(n: int) -> np.ndarray:
    """eq. (kj): k_j = -pi + 2 (j-1) pi / n_k, j = 1..n_k (returned 0-based)."""
    return -np.pi + 2.0 * np.pi * np.arange(n) / n


def allind_kpk(j1: int, j2: int, nk: int) -> int:
    """1-based index of k_{j1} + k_{j2} (three cases of the paper's formula)."""
    k = kgrid(nk)
    s = k[j1 - 1] + k[j2 - 1]
    if s < -np.pi - 1e-12:
        return j1 + j2 + nk // 2 - 1
    if s < np.pi - 1e-12:
        return j1 + j2 - nk // 2 - 1
    return j1 + j2 - 3 * nk // 2 - 1


def allind_kmk(j1: int, j2: int, nk: int) -> int:
    """1-based index of k_{j1} - k_{j2} (the paper's companion formula)."""
    k = kgrid(nk)
    s = k[j1 - 1] - k[j2 - 1]
    if s < -np.pi - 1e-12:
        return j1 - j2 + 3 * nk // 2 + 1
    if s < np.pi - 1e-12:
        return j1 - j2 + nk // 2 + 1
    return j1 - j2 - nk // 2 + 1


def backward(G: np.ndarray) -> np.ndarray:
    """G(k; t', t) = -[G(k; t, t')]^dag on the trailing two (band) axes."""
    return -np.conj(np.swapaxes(G, -1, -2))


def paper_sigma_direct(Gl: np.ndarray, Gg: np.ndarray, U: float, lesser: bool = True) -> np.ndarray:
    """Sigma^<_{jm}(k; t, t') of eq. (2BSE) by direct summation over q and k'.

    Gl, Gg: (nk, 2, 2) arrays G^<(k; t, t') and G^>(k; t, t') for the two bands.
    For Sigma^> (lesser=False) the roles of < and > are swapped, as the paper
    states ("similar expressions").
    """
    nk = Gl.shape[0]
    A = Gl if lesser else Gg          # forward-line propagators G^{</>}(t, t')
    B = backward(Gg if lesser else Gl)  # backward line G^{>/<}(t', t)
    out = np.zeros((nk, 2, 2), complex)
    bar = {0: 1, 1: 0}
    for kk in range(1, nk + 1):
        for j in range(2):
            for m in range(2):
                jb, mb = bar[j], bar[m]
                s = 0.0
                for q in range(1, nk + 1):
                    kmq = allind_kmk(kk, q, nk)
                    for kp in range(1, nk + 1):
                        kpq = allind_kpk(kp, q, nk)
                        # direct term: G_{jb mb}(k'+q) G_{mb jb}(k'; t', t) G_{jm}(k-q)
                        s += A[kpq - 1, jb, mb] * B[kp - 1, mb, jb] * A[kmq - 1, j, m]
                        # exchange term: G_{j mb}(k') G_{mb jb}(k'+q-k; t', t) G_{jb m}(q)
                        idx = allind_kmk(kpq, kk, nk)
                        s -= A[kp - 1, j, mb] * B[idx - 1, mb, jb] * A[q - 1, jb, m]
                out[kk - 1, j, m] = U * U * s / nk ** 2
    return out


def hubbard_sigma_direct(Gl: np.ndarray, Gg: np.ndarray, U: float, nkx: int, nky: int,
                         lesser: bool = True) -> np.ndarray:
    """Spin-degenerate intra-orbital Hubbard second Born as a momentum convolution:

    Sigma^<_ab(k; t,t') = U^2/N_k^2 sum_{k1,k2} G^<_ab(k1; t,t') G^<_ab(k2; t,t')
                                                G^>_ba(k1 + k2 - k; t', t).
    Gl, Gg: (nk, nb, nb), k flattened as ix * nky + iy.
    """
    nk, nb, _ = Gl.shape
    A = Gl if lesser else Gg
    B = backward(Gg if lesser else Gl)
    ix = np.arange(nk) // nky
    iy = np.arange(nk) % nky
    out = np.zeros((nk, nb, nb), complex)
    for k in range(nk):
        for k1 in range(nk):
            jx = (ix[k1] + ix - ix[k]) % nkx
            jy = (iy[k1] + iy - iy[k]) % nky
            k3 = jx * nky + jy           # index of k1 + k2 - k for every k2
            for a in range(nb):
                for b in range(nb):
                    out[k, a, b] += A[k1, a, b] * np.sum(A[:, a, b] * B[k3, b, a])
    return U * U * out / nk ** 2


def h0_numpy(hop: np.ndarray, nkx: int, nky: int, A: float, pol=(1.0, 0.0)) -> np.ndarray:
    """Bloch Hamiltonian T0 + sum_d (T_d e^{i q_d} + h.c.) at q = k - A pol."""
    kx = kgrid(nkx)
    ky = kgrid(nky)
    out = []
    for x in kx:
        for y in ky:
            qx, qy = x - A * pol[0], y - A * pol[1]
            h = hop[0] + hop[1] * np.exp(1j * qx) + hop[1].conj().T * np.exp(-1j * qx)
            if nky > 1:
                h = h + hop[2] * np.exp(1j * qy) + hop[2].conj().T * np.exp(-1j * qy)
            out.append(h)
    return np.array(out)


def tdhf_rk4(cfg, rho0: np.ndarray, T: float, nsub: int):
    """d rho_k/dt = -i [h0(k - A(t)) + Sigma^HF[rho], rho_k] by RK4 with step dt/nsub,
    Sigma^HF_ab = delta_ab U rho_loc,aa (Hubbard). Returns rho at t = 0, dt, 2dt, ..."""
    pu = cfg.pulse

    def A(t):
        return pu.amp * np.sin(pu.omega * t) * np.exp(-((t - pu.t0) / pu.width) ** 2)

    def rhs(t, r):
        loc = r.mean(axis=0)
        hf = np.diag(cfg.U * np.real(np.diag(loc))) if cfg.hf else 0.0
        h = h0_numpy(cfg.hop, cfg.nkx, cfg.nky, A(t), pu.pol) + hf
        return -1j * (h @ r - r @ h)

    h = cfg.dt / nsub
    nsteps = int(round(T / cfg.dt))
    r = rho0.copy()
    out = [r.copy()]
    t = 0.0
    for _ in range(nsteps):
        for _ in range(nsub):
            k1 = rhs(t, r)
            k2 = rhs(t + h / 2, r + h / 2 * k1)
            k3 = rhs(t + h / 2, r + h / 2 * k2)
            k4 = rhs(t + h, r + h * k3)
            r = r + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
            t += h
        out.append(r.copy())
    return np.array(out)
