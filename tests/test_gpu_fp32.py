"""The FP32 forms of the history sums (history stored in complex64, products and tile
accumulation in FP32, everything else FP64), against the FP64 oracle: the vector-ALU form
(KBE_FP32) and the matrix-core form (KBE_FP32_MFMA: quad layout, column sums on
v_mfma_f32_16x16x4f32 with the self-energy split into FP32 high and low parts).

Tolerances: the propagated observables must stay within 1e-6 relative of the FP64
oracle (per series, normalised by the series' largest magnitude). For one history pass
on random inputs the bound follows from FP32 arithmetic: each product carries 2^-24
relative rounding (Sigma is rounded to FP32 too) and the sums run over up to ~10^2
terms per tile with random signs, so the error stays below ~10^-6 of the largest
output; 1e-5 leaves a margin of ten.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2505_19467_amd import inputs

pytestmark = pytest.mark.gpu

PASS_TOL = 1e-5
RUN_TOL = 1e-6


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2505_19467_amd import kbe
    return kbe


def _rel(got, ref):
    return np.abs(np.asarray(got) - np.asarray(ref)).max() / np.abs(ref).max()


FORMS = [inputs.PRECISION_FP32, inputs.PRECISION_FP32_MFMA]
FORM_ID = {inputs.PRECISION_FP32: "valu", inputs.PRECISION_FP32_MFMA: "mfma"}


@pytest.mark.parametrize("prec", FORMS, ids=FORM_ID.get)
@pytest.mark.parametrize("nkx,nky,nb,m", [(3, 2, 2, 130), (2, 2, 1, 70), (2, 1, 3, 66), (1, 2, 2, 1), (2, 1, 2, 17),
                                          (2, 1, 2, 129), (1, 2, 1, 257), (1, 1, 4, 129), (2, 1, 2, 64),
                                          (1, 1, 4, 70), (2, 1, 2, 203)])
def test_fp32_collision_row(K, nkx, nky, nb, m, prec):
    import torch
    _say(f"fp32 collision ({FORM_ID[prec]}) nk={nkx}x{nky} nb={nb} m={m}")
    hop = np.zeros((3, nb, nb), complex)
    cfg = inputs.Config(name="t", nkx=nkx, nky=nky, nb=nb, hop=hop, U=1.0, dt=0.02, nt=m + 2,
                        precision=prec)
    S = K.System(cfg)
    assert S.history.dtype == torch.complex64
    rows = [r.astype(np.complex64).astype(np.complex128) for r in inputs.random_history(cfg.nk, nb, m, seed=3 + m)]
    sig = inputs.random_complex((m + 1, cfg.nk, 2, nb, nb), 5 + m, scale=0.4)
    for j in range(m + 1):
        S.set_history_row(j, torch.from_numpy(rows[j]).cuda())
    dst = S.sigma_planes()
    t = torch.from_numpy(sig).cuda().reshape(m + 1, cfg.nk, 2, nb * nb).permute(1, 2, 3, 0)
    dst[:, :2, :, :m + 1].copy_(t)
    dst[:, 2, :, :m + 1].copy_(t[:, 1] - t[:, 0])
    S.rebuild_aux(m)
    S.stage_collision(m)
    got = S.collision_row(m).cpu().numpy()
    ref = O.collision_row(cfg, m, rows, sig)
    err = _rel(got, ref)
    _say(f"  relative error {err:.2e}")
    assert err < PASS_TOL


@pytest.mark.parametrize("prec", FORMS, ids=FORM_ID.get)
@pytest.mark.parametrize("name,ks", [("c2", (0, 313, 575)), ("c5", (0, 129, 255))])
def test_fp32_collision_full_size_sampled(K, name, ks, prec):
    """The FP32-form history sums at the full workload sizes (24x24, nb = 2, m = 1000 and
    16x16, nb = 4, m = 1600: 87 GB of complex64), in the launch configuration the benchmark
    times; sampled k-points recomputed by the oracle from the stored FP32 blocks."""
    from tests.sampled import collision_reference
    import torch
    cfg = inputs.WORKLOADS[name]().replace(precision=prec)
    m = cfg.nt
    _say(f"full-size fp32 collision ({FORM_ID[prec]}) {name} m={m} nk={cfg.nk} nb={cfg.nb}")
    S = K.System(cfg)
    assert S.history.dtype == torch.complex64
    inputs.fill_normal_(S.history, seed=31, scale=0.3)
    inputs.fill_normal_(S.sigma_planes(), seed=32, scale=0.3)
    sp = S.sigma_planes()
    sp[:, 2].copy_(sp[:, 1] - sp[:, 0])
    S.rebuild_aux(m)
    S.stage_collision(m)
    got_all = S.collision_row(m).cpu().numpy()
    sig_all = S.sigma_row(m).cpu().numpy()
    for k in ks:
        ref = collision_reference(K, S, cfg, m, k, sig_all)
        err = _rel(got_all[:, k:k + 1], ref)
        _say(f"  k={k}: relative error {err:.2e}")
        assert err < PASS_TOL
    S.close()
    del S


SERIES = ["N", "Ekin", "EHF", "Ecorr", "Etot", "Jx", "n_orb0", "n_orb1", "n_band0", "n_band1"]


@pytest.mark.parametrize("prec", FORMS, ids=FORM_ID.get)
@pytest.mark.parametrize("name,nsteps", [("c1", 200), ("c4", 60), ("c2", 40), ("c5", 70)])
def test_fp32_run_accuracy(K, name, nsteps, prec):
    _say(f"fp32 run ({FORM_ID[prec]}) {name} steps={nsteps}")
    cfg = inputs.WORKLOADS[name]().replace(precision=prec)
    S = K.System(cfg, nt_max=nsteps)
    S.step(nsteps)
    obs = S.observables()
    ref = O.run(cfg.replace(precision=inputs.PRECISION_FP64), nsteps)["obs"]
    errs = {n: _rel(obs[:, O.OBS[n]], ref[:, O.OBS[n]]) for n in SERIES}
    _say("  " + " ".join(f"{k}={v:.1e}" for k, v in errs.items()))
    bad = {k: v for k, v in errs.items() if not v < RUN_TOL}
    assert not bad, bad
    # the FP32 form must not be bit-identical to FP64 (it really runs in FP32)
    assert max(errs.values()) > 0.0


@pytest.mark.parametrize("nkx,nky,nb,nsteps", [(5, 3, 3, 70), (7, 1, 1, 90), (3, 3, 4, 75)])
def test_fp32_mfma_run_shapes(K, nkx, nky, nb, nsteps):
    """The matrix-core form on the other orbital counts (nb = 1, 3, 4) and odd grids, past the
    first strip, against the FP64 oracle."""
    _say(f"fp32 mfma run shape {nkx}x{nky} nb={nb} steps={nsteps}")
    rng = np.random.default_rng(40 + nb)
    hop = np.zeros((3, nb, nb), complex)
    hop[0] = inputs.random_hermitian(nb, 1, 41 + nb)[0]
    hop[1] = -(np.eye(nb) + 0.2 * rng.standard_normal((nb, nb)))
    hop[2] = -(0.7 * np.eye(nb) + 0.1 * rng.standard_normal((nb, nb))) if nky > 1 else 0
    cfg = inputs.Config(name=f"mfma_{nkx}x{nky}_nb{nb}", nkx=nkx, nky=nky, nb=nb, hop=hop, U=1.2, dt=0.03,
                        nt=nsteps, precision=inputs.PRECISION_FP32_MFMA,
                        pulse=inputs.Pulse(amp=0.7, omega=1.3, t0=0.3, width=0.8, pol=(0.8, 0.6)))
    S = K.System(cfg)
    S.step(nsteps)
    obs = S.observables()
    ref = O.run(cfg.replace(precision=inputs.PRECISION_FP64), nsteps)["obs"]
    errs = {}
    for n in SERIES:
        r = ref[:, O.OBS[n]]
        if np.abs(r).max() > 1e-12:
            errs[n] = _rel(obs[:, O.OBS[n]], r)
    _say("  " + " ".join(f"{k}={v:.1e}" for k, v in errs.items()))
    bad = {k: v for k, v in errs.items() if not v < RUN_TOL}
    assert not bad, bad
    S.close()
