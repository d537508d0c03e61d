"""kbe_create_noalloc (the workspace in the library's static per-device array) against
kbe_create on caller-owned buffers: two contexts in a row, the second smaller, each propagated
and compared with the same run on a kbe_create context. The kernels and their inputs are the
same, so the observables and the history rows must agree bit for bit (stricter than the 1e-10
relative FP64 bar)."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2505_19467_amd import inputs

pytestmark = pytest.mark.gpu


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


def _run(K, cfg, n, noalloc):
    S = K.System(cfg, nt_max=n, noalloc=noalloc)
    S.step(n)
    obs = S.observables()
    rows = [S.history_row(j).cpu().numpy() for j in (0, n // 2, n)]
    S.close()
    return obs, rows


def test_noalloc_matches_kbe_create_twice(K):
    cases = [(inputs.c1(), 60), (inputs.c1().replace(nkx=8, n_corr=2), 30)]
    sizes = []
    for cfg, n in cases:
        _, wb, _ = K.workspace_query(cfg, n)
        sizes.append(wb)
        assert wb <= K.NOALLOC_WORKSPACE_MAX
        _say(f"no-alloc: {cfg.name} nk={cfg.nk} K={cfg.n_corr} steps={n} workspace {wb} B")
        ref_obs, ref_rows = _run(K, cfg, n, noalloc=False)
        obs, rows = _run(K, cfg, n, noalloc=True)
        assert np.array_equal(obs, ref_obs)
        for r, rr in zip(rows, ref_rows):
            assert np.array_equal(r, rr)
    assert sizes[1] < sizes[0]   # the second context is the smaller one


def test_noalloc_refusals(K):
    """A workload whose workspace exceeds the static array is refused before any launch, and a
    device holds one allocation-free context at a time."""
    import torch
    cfg = inputs.c2()
    _, wb, _ = K.workspace_query(cfg)
    assert wb > K.NOALLOC_WORKSPACE_MAX
    c = K._c_config(cfg)
    p = K.KbePulse()
    hop = np.ascontiguousarray(cfg.hop, np.complex128).view(np.float64)
    ctx = ctypes.c_void_p()
    dummy = torch.empty(256, dtype=torch.uint8, device="cuda")
    rc = K._lib.kbe_create_noalloc(ctypes.byref(c), hop.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   ctypes.byref(p), ctypes.c_void_p(dummy.data_ptr()), 1 << 62,
                                   ctypes.c_void_p(dummy.data_ptr()), 1 << 62, None, ctypes.byref(ctx))
    assert rc == -2 and not ctx.value           # KBE_ERR_SHAPE
    small = inputs.c1()
    A = K.System(small, nt_max=10, noalloc=True)
    with pytest.raises(K.KbeError, match="KBE_ERR_STATE"):
        K.System(small, nt_max=10, noalloc=True)
    A.step(3)
    A.close()
    B = K.System(small, nt_max=10, noalloc=True)   # free again once the first is destroyed
    B.step(3)
    got = B.observables()
    B.close()
    R = K.System(small, nt_max=10)
    R.step(3)
    assert np.array_equal(got, R.observables())
    R.close()
