"""Full-length trajectories of the HIP path against stored CPU-oracle values.

The files under tests/golden/ were written by ``tests/golden/make_goldens.py``, which calls only
the oracle (the 24x24 run takes hours on the CPU, so it is stored, not recomputed here):

* the 24x24, nb = 2 workload propagated for all 1000 steps (Algorithm "prop", K = 1): every
  observable series and sampled entries of the final row G(t_1000, .), against the FP64 path
  (1e-10 relative, the FP64 target) and both FP32-storage forms (1e-6 relative);
* the paper's own model on the chain of n_k = 1024 points (interband U, the dipole kick at
  step 25) for its first 100 steps, against the FP64 path (1e-10);
* the 12x12 gradient workload at its full 400 steps: the oracle's tangent-linear derivatives
  of the final upper-band occupation, against the reverse sweep (1e-9 relative).

Series that vanish by symmetry (J_y for a pulse along x) are compared in absolute terms: both
sides must stay at the rounding level of the O(1) terms that cancel (1e-14).
"""
import os
import sys

import numpy as np
import pytest

from paper_2505_19467_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FP64_TOL = 1e-10
FP32_TOL = 1e-6
TLM_TOL = 1e-9
VANISH = 1e-12      # a reference series below this vanishes by symmetry
VANISH_BOUND = 1e-14


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


def _load_table(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} has not been written yet (tests/golden/make_goldens.py)")
    cols = None
    with open(path) as f:
        for line in f:
            if line.startswith("# columns:"):
                cols = line.split(":", 1)[1].split()
    return cols, np.loadtxt(path, comments="#")


def _golden_run(prefix):
    cols, obs = _load_table(f"{prefix}_obs.txt")
    _, fr = _load_table(f"{prefix}_final_row.txt")
    return cols, obs, fr


def _compare_c2(K, cfg, tol):
    _compare_run(K, cfg, cfg.nt, "c2_nt1000", tol)


def _compare_run(K, cfg, n, prefix, tol):
    cols, gobs, gfr = _golden_run(prefix)
    assert gobs.shape[0] == n + 1
    S = K.System(cfg, nt_max=n)
    S.step(n)
    obs = S.observables()
    final = S.history_row(n).cpu().numpy()       # [t'][k][comp][a][b]
    S.close()
    worst = {}
    vanish = {}
    for j, name in enumerate(cols):
        x, r = obs[:, K.OBS[name]], gobs[:, j]
        if name == "t":
            assert np.abs(x - r).max() < 1e-12
            continue
        if np.abs(r).max() < VANISH:
            vanish[name] = float(np.abs(x).max())
            assert vanish[name] < VANISH_BOUND, name
            continue
        worst[name] = float(np.abs(x - r).max() / np.abs(r).max())
    k, tp, c, a, b = (gfr[:, i].astype(int) for i in range(5))
    ref = gfr[:, 5] + 1j * gfr[:, 6]
    got = final[tp, k, c, a, b]
    worst["final_row"] = float(np.abs(got - ref).max() / np.abs(ref).max())
    _say(f"  {cfg.name} {n} steps vs oracle: worst {max(worst.values()):.2e} " +
         " ".join(f"{kk}={v:.1e}" for kk, v in worst.items()) +
         "; vanishing series " + " ".join(f"{kk}={v:.1e}" for kk, v in vanish.items()))
    bad = {kk: v for kk, v in worst.items() if not v < tol}
    assert not bad, bad


def test_c2_full_run_fp64_matches_oracle(K):
    _say("golden: 24x24 nb=2 FP64, 1000 steps")
    _compare_c2(K, inputs.c2(), FP64_TOL)


def test_c2_full_run_fp32_form_matches_oracle(K):
    _say("golden: 24x24 nb=2 FP32 form, 1000 steps")
    _compare_c2(K, inputs.c2().replace(precision=inputs.PRECISION_FP32), FP32_TOL)


def test_c2_full_run_fp32_mfma_form_matches_oracle(K):
    _say("golden: 24x24 nb=2 FP32-MFMA form, 1000 steps")
    _compare_c2(K, inputs.c3(), FP32_TOL)


def test_paper_model_100_steps_matches_oracle(K):
    """The paper's workload at its n_k = 1024 through the dipole kick (step 25) and 75 steps
    beyond it."""
    _say("golden: chain n_k = 1024, interband U, dipole kick, FP64, 100 steps")
    _compare_run(K, inputs.paper_chain(), 100, "p1_nt100", FP64_TOL)


def test_c4_full_gradient_matches_tangent_linear_oracle(K):
    """The gradient workload at its full length: d n_band1(t_400) / d(amp, omega, U)."""
    _say("golden: 12x12 nb=2 reverse sweep over 400 steps vs the tangent-linear oracle")
    _, tab = _load_table("c4_nt400_tlm.txt")
    cfg = inputs.c4()
    n = cfg.nt
    assert tab.shape[0] == n + 1
    S = K.System(cfg)
    S.step(n)
    val = S.observables(n, 1)[0, K.OBS["n_band1"]]
    g = S.adjoint_gradient("n_band1")
    S.close()
    ref_val, ref = tab[n, 1], tab[n, 2:5]
    err = np.abs(g - ref).max() / np.abs(ref).max()
    _say(f"  n_band1(T) {val:.15f} (oracle {ref_val:.15f}); grad {g} oracle {ref}; rel err {err:.2e}")
    assert abs(val - ref_val) <= FP64_TOL * max(1.0, abs(ref_val))
    assert err <= TLM_TOL
