"""The corrector's stopping rule of Algorithm "prop" (at most n_corr passes, stop once the row
changes by at most corr_tol) on the GPU against the oracle's run with the same rule.

Both sides take the stop decision in FP64 on their own change values, which agree to ~1e-15
relative; the tolerances used here sit at least a factor 3 away from every change the oracle
logs, so the decisions cannot differ (checked in each test before the comparison). The
observables must then agree to 1e-10 relative (the FP64 target) and the passes exactly.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2505_19467_amd import inputs

pytestmark = pytest.mark.gpu

RUN_TOL = 1e-10
SERIES = ["N", "Ekin", "EHF", "Ecorr", "Etot", "Jx", "n_orb0", "n_orb1", "n_band0", "n_band1"]


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


def _series_err(obs, ref):
    worst = 0.0
    for name in SERIES:
        i = O.OBS[name]
        scale = np.abs(ref[:, i]).max()
        if scale < 1e-12:
            assert np.abs(obs[:, i]).max() < 1e-12, name
            continue
        worst = max(worst, np.abs(obs[:, i] - ref[:, i]).max() / scale)
    return worst


# tolerances in wide gaps of the changes the oracle logs for these runs (factors 8-18 away)
@pytest.mark.parametrize("name,n_corr,tol,nsteps", [("c1", 5, 1.7e-9, 60), ("c1", 6, 2.2e-6, 80),
                                                    ("c4", 4, 1.5e-8, 30), ("c2", 4, 6e-9, 20),
                                                    ("c5", 4, 6e-6, 20)])
def test_tolerance_corrector_matches_oracle(K, name, n_corr, tol, nsteps):
    _say(f"tolerance corrector {name} n_corr={n_corr} tol={tol:g} steps={nsteps}")
    cfg = inputs.WORKLOADS[name]().replace(n_corr=n_corr, corr_tol=tol)
    ref_obs, ref_passes, ref_ch = O.run_log(cfg, nsteps)
    logged = ref_ch[ref_ch > 0]
    margin = np.min(np.abs(np.log(logged / tol)))
    assert margin > np.log(3.0), f"tolerance {tol:g} within a factor 3 of a change: pick another"
    S = K.System(cfg, nt_max=nsteps)
    S.step(nsteps)
    obs = S.observables()
    passes, ch = S.corrector_log()
    _say(f"  passes per step: {np.bincount(passes[1:])}; oracle {np.bincount(ref_passes[1:])}")
    assert np.array_equal(passes, ref_passes)
    taken = ref_ch > 0
    assert np.array_equal(ch[1:] > 0, taken)
    # a change is the difference of two iterates of O(1) row entries: it carries their absolute
    # rounding (~1e-16 each, a few dozen operations deep), not a relative error of its own size
    chg_err = np.max(np.abs(ch[1:][taken] - ref_ch[taken]))
    err = _series_err(obs, ref_obs)
    _say(f"  observables: worst relative error {err:.2e}; row changes agree to {chg_err:.1e} (absolute)")
    assert err < RUN_TOL
    assert chg_err < 1e-13


def test_tolerance_limits_reproduce_fixed_counts(K):
    """corr_tol = 0 is the fixed-count corrector (bit for bit), a tolerance above every change
    stops after one pass (bit for bit the single-pass run)."""
    cfg = inputs.c1()
    n = 30
    runs = {}
    for key, c in (("fixed3", cfg.replace(n_corr=3)), ("tol0", cfg.replace(n_corr=3, corr_tol=0.0)),
                   ("fixed1", cfg.replace(n_corr=1)), ("tolinf", cfg.replace(n_corr=3, corr_tol=1e30))):
        S = K.System(c, nt_max=n)
        S.step(n)
        runs[key] = (S.observables(), S.history_row(n).cpu().numpy(), S.corrector_log()[0])
        S.close()
    assert np.array_equal(runs["fixed3"][0], runs["tol0"][0]) and np.array_equal(runs["fixed3"][1], runs["tol0"][1])
    assert np.array_equal(runs["fixed1"][0], runs["tolinf"][0]) and np.array_equal(runs["fixed1"][1], runs["tolinf"][1])
    assert np.all(runs["fixed3"][2][1:] == 3) and np.all(runs["tolinf"][2][1:] == 1)


def test_adjoint_refuses_tolerance_mode(K):
    cfg = inputs.c1().replace(corr_tol=1e-2, n_corr=1)   # a tolerance every step meets
    S = K.System(cfg, nt_max=5)
    S.step(3)
    with pytest.raises(K.KbeError):
        S.adjoint_gradient("n_band1")
    S.close()


@pytest.mark.parametrize("tol,nsteps", [(1e-30, 12), (1e-7, 40)])
def test_unmet_tolerance_reports_not_converged(K, tol, nsteps):
    """A step whose n_corr passes all end above corr_tol is committed and reported
    (KBE_ERR_NOT_CONVERGED): kbe_step stops on it, and stepping on continues the run. The
    flagged steps are the oracle's, the run matches the oracle's run with the same rule."""
    _say(f"unmet tolerance: c1 n_corr=2 tol={tol:g} steps={nsteps}")
    cfg = inputs.c1().replace(n_corr=2, corr_tol=tol)
    ref_obs, ref_passes, ref_ch, ref_unconv = O.run_log(cfg, nsteps, with_unconverged=True)
    # every logged change sits far (in absolute terms) from the tolerance compared with the
    # 1e-13 the two sides' changes agree to, so both take the same decisions
    assert np.min(np.abs(ref_ch[ref_ch > 0] - tol)) > 1e-11
    S = K.System(cfg, nt_max=nsteps)
    flagged, calls = [], 0
    while S.current_step < nsteps:
        calls += 1
        try:
            S.step(nsteps - S.current_step)
        except K.KbeNotConverged as e:
            assert e.step == S.current_step
            flagged.append(e.step)
    obs = S.observables()
    passes, _ = S.corrector_log()
    want = [int(m) for m in np.nonzero(ref_unconv)[0]]
    _say(f"  flagged {len(flagged)} of {nsteps} steps in {calls} calls; oracle {len(want)}")
    assert flagged == want and len(want) > 0
    assert np.array_equal(passes, ref_passes)
    assert _series_err(obs, ref_obs) < RUN_TOL
    S.close()
