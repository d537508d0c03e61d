"""Seeded synthetic inputs for the Kadanoff-Baym propagation step.

This module is the only code that both the HIP path's tests and the CPU oracle
consume. It holds parameter sets (lattice, hoppings, interaction, pulse, time
grid) and seeded random arrays, and none of the method's arithmetic: no
Hamiltonian, no self-energy, no collision integral, no time stepping.

Model family (two-band Hubbard model of Sec. "Computational Kernels", eq. (ham)
and (Green); the configurations below use its spin-degenerate on-site Hubbard
variant with a Peierls pulse, see the design notes):

* ``hop[0]`` is the on-site block T0, ``hop[1]`` the nearest-neighbour block
  along x, ``hop[2]`` along y (zero in 1D). All are complex nb x nb.
* The pulse is A(t) = amp * sin(omega * t) * exp(-((t - t0) / width)**2) along
  the unit vector ``pol`` (Peierls kind), or the dipole pulse of eq. (dipole),
  E(t) = amp * delta(t - t0) between bands 0 and 1 with d_k = 1 (dipole-kick kind).
"""
from __future__ import annotations

import dataclasses
import json
from dataclasses import dataclass, field

import numpy as np

INTERACTION_HUBBARD = 0   # spin-degenerate, intra-orbital on-site U (opposite spin only)
INTERACTION_INTERBAND = 1  # the paper's spinless two-band model, eq. (ham) / eq. (2BSE)

PULSE_PEIERLS = 0      # vector potential A(t) in the Bloch Hamiltonian
PULSE_DIPOLE_KICK = 1  # eq. (dipole): E(t) = amp * delta(t - t0), d_k = 1 (nb = 2)

PRECISION_FP64 = 0
PRECISION_FP32 = 1        # history stored and summed in FP32 on the vector ALU
PRECISION_FP32_MFMA = 2   # history stored in FP32, column sums on the matrix cores (hi/lo split Sigma)


@dataclass
class Pulse:
    amp: float = 0.5
    omega: float = 1.5
    t0: float = 2.0
    width: float = 1.0
    pol: tuple = (1.0, 0.0)
    kind: int = PULSE_PEIERLS


@dataclass
class Config:
    """One propagation workload. ``nky == 1`` means a 1D chain."""
    name: str
    nkx: int
    nky: int
    nb: int
    hop: np.ndarray                     # (3, nb, nb) complex128
    U: float
    dt: float
    nt: int
    pulse: Pulse = field(default_factory=Pulse)
    spin_deg: int = 2
    interaction: int = INTERACTION_HUBBARD
    hf: int = 1                         # include the first-order (Hartree-Fock) self-energy
    corr: int = 1                       # include the second-Born correlation self-energy
    n_corr: int = 1                     # corrector passes K per step (the maximum when corr_tol > 0)
    corr_tol: float = 0.0               # > 0: stop the corrector once the row changes by <= corr_tol
    quad_points: int = 1                # collision-integral quadrature: 1 = trapezoid, q > 1 = Gregory
                                        # end corrections on q nodes per end
    temp: float = 0.1
    filling: float = 0.5                # electrons per orbital per spin
    precision: int = PRECISION_FP64

    @property
    def dim(self) -> int:
        return 1 if self.nky == 1 else 2

    @property
    def nk(self) -> int:
        return self.nkx * self.nky

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)

    def to_json(self) -> str:
        d = dataclasses.asdict(self)
        d["hop"] = [[[[z.real, z.imag] for z in row] for row in blk] for blk in self.hop]
        return json.dumps(d, indent=1)


def _chain_hop(t11, t22, t12, e1, e2, two_d):
    hop = np.zeros((3, 2, 2), complex)
    hop[0] = np.diag([e1, e2])
    tx = -np.array([[t11, t12], [t12, t22]], complex)
    hop[1] = tx
    if two_d:
        hop[2] = tx
    return hop


def draw_c2_parameters(seed: int = 20250519):
    """Hoppings, on-site energies and U drawn uniformly within +-10% of nominal."""
    rng = np.random.default_rng(seed)
    nominal = np.array([1.0, 1.0, 0.3, 0.5, -0.5, 1.5])
    vals = nominal * rng.uniform(0.9, 1.1, size=6)
    t11, t22, t12, e1, e2, U = (float(v) for v in vals)
    return dict(t11=t11, t22=t22, t12=t12, e1=e1, e2=e2, U=U)


def haar_unitary(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random unitary from the QR factorisation of a complex Gaussian matrix,
    with the phases of R's diagonal moved into Q (Mezzadri's recipe)."""
    z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))


def c1() -> Config:
    """1D chain, nk=16, nb=2, U=1, dt=0.02, nt=200 (CPU oracle workload)."""
    return Config(name="c1_chain16_nb2", nkx=16, nky=1, nb=2,
                  hop=_chain_hop(1.0, 1.0, 0.3, 0.5, -0.5, False),
                  U=1.0, dt=0.02, nt=200)


def c2() -> Config:
    """2D square lattice, 24x24 k-grid, nb=2, seeded +-10% parameters, dt=0.02, nt=1000."""
    p = draw_c2_parameters()
    return Config(name="c2_sq24_nb2", nkx=24, nky=24, nb=2,
                  hop=_chain_hop(p["t11"], p["t22"], p["t12"], p["e1"], p["e2"], True),
                  U=p["U"], dt=0.02, nt=1000)


def c3() -> Config:
    """C2 with the history sums in the FP32 split-precision matrix-core form."""
    return c2().replace(name="c3_sq24_nb2_fp32mfma", precision=PRECISION_FP32_MFMA)


def c4() -> Config:
    """2D 12x12, nb=2, C2's parameter draw, dt=0.025, nt=400 (gradient workload)."""
    p = draw_c2_parameters()
    return Config(name="c4_sq12_nb2", nkx=12, nky=12, nb=2,
                  hop=_chain_hop(p["t11"], p["t22"], p["t12"], p["e1"], p["e2"], True),
                  U=p["U"], dt=0.025, nt=400)


def c5(seed: int = 20250520) -> Config:
    """2D 16x16, nb=4, random Hermitian on-site block with eigenvalues in [-2, 2]."""
    rng = np.random.default_rng(seed)
    lam = rng.uniform(-2.0, 2.0, size=4)
    q = haar_unitary(4, rng)
    hop = np.zeros((3, 4, 4), complex)
    hop[0] = q @ np.diag(lam) @ q.conj().T
    hop[0] = 0.5 * (hop[0] + hop[0].conj().T)
    tx = -(1.0 * np.eye(4) + 0.3 * (np.ones((4, 4)) - np.eye(4))).astype(complex)
    hop[1] = tx
    hop[2] = tx
    return Config(name="c5_sq16_nb4", nkx=16, nky=16, nb=4, hop=hop, U=2.0,
                  dt=0.015, nt=1600)


def paper_chain(nk: int = 1024, nt: int = 500) -> Config:
    """The paper's model problem (Sec. "Computational Kernels"): a spinless two-band chain with
    the band energies eps_v = -2(1 - cos k) - Eg/2 and eps_c = 2(1 - cos k) + Eg/2 (Eg = 1), the
    interband interaction of eq. (ham) with its -U n_c term, and the dipole pulse of
    eq. (dipole), E(t) = I delta(t - 0.5) with d_k = 1; n_k = 1024 and a 500-step history as in
    the paper's timing runs. U = 1, I = 0.25, dt = 0.02 and T = 0.1 (valence band filled) are
    not given by the paper."""
    eg = 1.0
    hop = np.zeros((3, 2, 2), complex)
    hop[0] = np.diag([-2.0 - eg / 2, 2.0 + eg / 2])
    hop[1] = np.diag([1.0, -1.0])
    return Config(name=f"p1_chain{nk}_interband", nkx=nk, nky=1, nb=2, hop=hop, U=1.0, dt=0.02, nt=nt,
                  pulse=Pulse(amp=0.25, omega=0.0, t0=0.5, width=1.0, pol=(1.0, 0.0), kind=PULSE_DIPOLE_KICK),
                  spin_deg=1, interaction=INTERACTION_INTERBAND)


WORKLOADS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5, "p1": paper_chain}


# ----------------------------------------------------------------------------
# Seeded random arrays (for kernel-level checks). Plain random numbers only.
# ----------------------------------------------------------------------------

def random_complex(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def random_history(nk: int, nb: int, m: int, seed: int, scale: float = 0.3):
    """Rows 0..m of a two-time lower triangle, as a list of arrays: row j has shape
    (j+1, nk, 2, nb, nb) = [t'][k][lesser/greater][a][b]."""
    rng = np.random.default_rng(seed)
    rows = []
    for j in range(m + 1):
        shp = (j + 1, nk, 2, nb, nb)
        rows.append(scale * (rng.standard_normal(shp) + 1j * rng.standard_normal(shp)))
    return rows


def random_hermitian(n: int, count: int, seed: int, scale: float = 1.0) -> np.ndarray:
    z = random_complex((count, n, n), seed, scale)
    return 0.5 * (z + np.conj(np.swapaxes(z, -1, -2)))


def fill_normal_(tensor, seed: int, scale: float = 1.0):
    """Fill a (real or complex) torch tensor in place with seeded standard-normal numbers,
    on the tensor's own device (torch's generator; used for full-size synthetic histories)."""
    import torch
    g = torch.Generator(device=tensor.device)
    g.manual_seed(seed)
    view = torch.view_as_real(tensor) if tensor.is_complex() else tensor
    view.normal_(0.0, scale, generator=g)
    return tensor
