"""The paper's own model on the GPU against the oracle: the interband second-Born self-energy
of eq. (2BSE) (direct minus exchange) with its -U n_c term and Hartree-Fock field, the dipole
delta pulse of eq. (dipole), and chains of up to 1024 k-points (the paper's n_k), through the
C ABI. Tolerances as in the FP64 parity tests: single stages <= 1e-12, propagations <= 1e-10
relative; the FP32 form <= 1e-6 against the FP64 oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2505_19467_amd import inputs
from tests.test_gpu_parity import KERNEL_TOL, _compare_run, _say, relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2505_19467_amd import kbe
    return kbe


def _interband(nkx, nky, nt, **kw):
    cfg = inputs.paper_chain(nk=nkx, nt=nt).replace(nky=nky, **kw)
    if nky > 1:
        hop = cfg.hop.copy()
        hop[2] = hop[1]
        cfg = cfg.replace(hop=hop)
    return cfg


def _sigma_case(K, cfg, m, seed):
    import torch
    S = K.System(cfg)
    row = inputs.random_complex((m + 1, cfg.nk, 2, cfg.nb, cfg.nb), seed, scale=0.5)
    S.set_history_row(m, torch.from_numpy(row).cuda())
    S.rebuild_aux(m)
    S.stage_sigma(m)
    return S, row


# chains: 16 (compile-time transform), 37 (prime: direct line sums), 96 (8 x 12 split), 200 (10 x 20:
# more than 8 first-stage outputs per line), 128 / 512 (power-of-two FFT with a radix-2 stage),
# 256 / 1024 (radix-4 stages only; 1024 is the paper's n_k); 2D grids
@pytest.mark.parametrize("nkx,nky,m", [(16, 1, 5), (37, 1, 4), (96, 1, 9), (200, 1, 3), (128, 1, 6),
                                       (256, 1, 4), (512, 1, 3), (1024, 1, 2),
                                       (4, 3, 7), (6, 4, 70), (5, 5, 0)])
def test_interband_sigma_row_parity(K, nkx, nky, m):
    _say(f"interband sigma nk={nkx}x{nky} m={m}")
    cfg = _interband(nkx, nky, m + 2)
    S, row = _sigma_case(K, cfg, m, 300 + m + nkx)
    got = S.sigma_row(m).cpu().numpy()
    ref = O.sigma_row(cfg, m, row)
    assert relerr(got, ref) < KERNEL_TOL
    sp = S.sigma_planes()[:, :, :, :m + 1].cpu().numpy()
    assert np.abs(sp[:, 2] - (sp[:, 1] - sp[:, 0])).max() <= 1e-15 * max(1.0, np.abs(sp).max())


@pytest.mark.parametrize("nkx,nb,m", [(1024, 2, 2), (200, 1, 5), (96, 2, 4)])
def test_hubbard_sigma_long_chains(K, nkx, nb, m):
    """The Hubbard preset's self-energy on chains longer than 64 points (the runtime transform)."""
    _say(f"hubbard sigma chain {nkx} nb={nb} m={m}")
    hop = np.zeros((3, nb, nb), complex)
    hop[0] = np.diag(np.linspace(-0.5, 0.5, nb))
    hop[1] = -np.eye(nb)
    cfg = inputs.Config(name="chain", nkx=nkx, nky=1, nb=nb, hop=hop, U=1.3, dt=0.02, nt=m + 2)
    S, row = _sigma_case(K, cfg, m, 400 + m + nkx)
    assert relerr(S.sigma_row(m).cpu().numpy(), O.sigma_row(cfg, m, row)) < KERNEL_TOL


def test_interband_sigma_full_size_sampled(K):
    """The interband self-energy at the paper's size (n_k = 1024, the slice at m = 500: 501
    times, the launch the benchmark times) on a seeded random row; sampled t_j recomputed by the
    oracle one pair at a time (Sigma(t_m, t_j) depends only on G(t_m, t_j))."""
    cfg = inputs.paper_chain()
    m = cfg.nt
    _say(f"full-size interband sigma nk={cfg.nk} m={m}")
    S, row = _sigma_case(K, cfg, m, 2028)
    got = S.sigma_row(m).cpu().numpy()
    for j in (0, 1, 250, m - 1, m):
        ref = O.sigma_row(cfg, 0, row[j:j + 1])
        err = relerr(got[j:j + 1], ref)
        _say(f"  t_j={j}: rel err {err:.2e}")
        assert err < KERNEL_TOL
    S.close()


@pytest.mark.parametrize("label,cfg,nsteps", [
    ("paper model, 16-point chain, kick at t = 0.5", _interband(16, 1, 60), 60),
    ("paper model, 64-point chain", _interband(64, 1, 40), 40),
    ("paper model, 200-point chain, kick at step 6", _interband(200, 1, 20, pulse=inputs.Pulse(
        amp=0.4, omega=0.0, t0=0.1, kind=inputs.PULSE_DIPOLE_KICK)), 20),
    ("paper model, K = 2 and Gregory q = 4", _interband(16, 1, 50, n_corr=2, quad_points=4), 50),
    ("interband 2D 4x4, Peierls pulse", _interband(4, 4, 30, pulse=inputs.Pulse(amp=0.6, omega=1.4, t0=0.3)), 30),
    ("Hubbard chain with the dipole kick", inputs.c1().replace(pulse=inputs.Pulse(
        amp=0.5, omega=0.0, t0=0.2, kind=inputs.PULSE_DIPOLE_KICK)), 40),
    ("paper model, kick at t = 0 (the first step)", _interband(16, 1, 20, pulse=inputs.Pulse(
        amp=0.3, omega=0.0, t0=0.0, kind=inputs.PULSE_DIPOLE_KICK)), 20),
])
def test_paper_model_run_parity(K, label, cfg, nsteps):
    _say(f"run parity: {label}, {nsteps} steps")
    _compare_run(K, cfg, nsteps)


def test_paper_model_run_parity_nk1024(K):
    """A propagation at the paper's n_k = 1024 through the kick (moved to t = 0.1 so that a few
    steps reach it)."""
    cfg = inputs.paper_chain(nt=10).replace(pulse=inputs.Pulse(amp=0.25, omega=0.0, t0=0.1,
                                                               kind=inputs.PULSE_DIPOLE_KICK))
    _say("run parity: paper model at n_k = 1024, 10 steps")
    _compare_run(K, cfg, 10)


def test_paper_model_fp32_form(K):
    cfg = _interband(64, 1, 80, precision=inputs.PRECISION_FP32)
    S = K.System(cfg, nt_max=80)
    S.step(80)
    obs = S.observables()
    ref = O.run(cfg.replace(precision=inputs.PRECISION_FP64), 80)["obs"]
    worst = 0.0
    for name in ("N", "Ekin", "EHF", "Ecorr", "Etot", "n_band0", "n_band1"):
        i = O.OBS[name]
        worst = max(worst, np.abs(obs[:, i] - ref[:, i]).max() / np.abs(ref[:, i]).max())
    _say(f"  FP32 form, paper model: worst relative deviation {worst:.2e}")
    assert 0.0 < worst < 1e-6


def test_adjoint_refuses_paper_model(K):
    S = K.System(_interband(16, 1, 10), nt_max=5)
    S.step(3)
    with pytest.raises(K.KbeError):
        S.adjoint_gradient("n_band1")
    S.close()


# ---------------------------------------------------------------- the paper's direct sums
@pytest.mark.parametrize("nkx,m", [(8, 0), (16, 3), (24, 4), (64, 5), (104, 2), (1024, 1)])
def test_sigma_direct_parity(K, nkx, m):
    """kbe_stage_sigma_direct (eq. (polarizability)/(kernel2) and Alg. "contraction2") gives the
    oracle's self-energy, and the transform route's to rounding."""
    _say(f"direct-sum sigma chain {nkx} m={m}")
    cfg = _interband(nkx, 1, m + 2)
    S, row = _sigma_case(K, cfg, m, 500 + m + nkx)
    fft = S.sigma_row(m).cpu().numpy()
    S.stage_sigma_direct(m)
    got = S.sigma_row(m).cpu().numpy()
    assert relerr(got, O.sigma_row(cfg, m, row)) < KERNEL_TOL
    assert relerr(got, fft) < KERNEL_TOL
    sp = S.sigma_planes()[:, :, :, :m + 1].cpu().numpy()
    assert np.abs(sp[:, 2] - (sp[:, 1] - sp[:, 0])).max() <= 1e-15 * max(1.0, np.abs(sp).max())


def test_sigma_direct_full_size(K):
    """The direct sums at the paper's size (n_k = 1024, the slice at m = 500: the call the
    benchmark times) against the transform route on every output, and against the oracle on
    sampled t_j."""
    cfg = inputs.paper_chain()
    m = cfg.nt
    _say(f"full-size direct-sum sigma nk={cfg.nk} m={m}")
    S, row = _sigma_case(K, cfg, m, 2029)
    fft = S.sigma_row(m).cpu().numpy()
    S.stage_sigma_direct(m)
    got = S.sigma_row(m).cpu().numpy()
    err = relerr(got, fft)
    _say(f"  direct vs transforms, all outputs: rel err {err:.2e}")
    assert err < KERNEL_TOL
    for j in (0, 333, m):
        e = relerr(got[j:j + 1], O.sigma_row(cfg, 0, row[j:j + 1]))
        _say(f"  t_j={j} vs oracle: rel err {e:.2e}")
        assert e < KERNEL_TOL
    S.close()


def test_sigma_direct_refuses_other_shapes(K):
    for cfg in (_interband(20, 1, 4), inputs.c1(), _interband(4, 4, 4)):
        S = K.System(cfg, nt_max=3)
        with pytest.raises(K.KbeError):
            S.stage_sigma_direct(0)
        S.close()


def test_stage_api_with_kick_composes_to_step(K):
    """With the dipole kick the stage entry points still reproduce kbe_step bit for bit: the
    commit of the kick slice applies the kick and evaluates the slice again."""
    cfg = _interband(16, 1, 12, pulse=inputs.Pulse(amp=0.4, omega=0.0, t0=0.1, kind=inputs.PULSE_DIPOLE_KICK))
    n = 10
    A = K.System(cfg, nt_max=n)
    A.step(n)
    B = K.System(cfg, nt_max=n)
    for m in range(1, n + 1):
        B.stage_propagators(m, 0)
        B.stage_update(m, 0)
        for _ in range(cfg.n_corr):
            B.stage_sigma(m)
            B.stage_collision(m)
            B.stage_propagators(m, 1)
            B.stage_update(m, 1)
        B.stage_sigma(m)
        B.stage_collision(m)
        B.stage_observables(m)
        B.stage_commit(m)
    assert np.array_equal(A.observables(), B.observables())
    assert np.array_equal(A.history_row(n).cpu().numpy(), B.history_row(n).cpu().numpy())
    assert np.array_equal(A.history_row(5).cpu().numpy(), B.history_row(5).cpu().numpy())


def test_adjoint_refuses_dipole_kick(K):
    """The reverse sweep covers the Peierls pulse only: a Hubbard context driven by the dipole
    kick is refused as well."""
    cfg = inputs.c1().replace(pulse=inputs.Pulse(amp=0.3, omega=0.0, t0=0.04, kind=inputs.PULSE_DIPOLE_KICK))
    S = K.System(cfg, nt_max=6)
    S.step(4)
    with pytest.raises(K.KbeError):
        S.adjoint_gradient("n_band1")
    S.close()
