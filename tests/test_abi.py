"""The C ABI: header declarations, exported symbols and the pure-host sizing call (CPU)."""
import ctypes
import os
import re

import pytest

from paper_2505_19467_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kbe.h")
LIB = os.path.join(ROOT, "paper_2505_19467_amd", "libkbe.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kbe_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("kbe_workspace_query", "kbe_create", "kbe_step", "kbe_observables", "kbe_destroy",
                     "kbe_last_error", "kbe_stage_sigma", "kbe_stage_collision", "kbe_stage_update",
                     "kbe_stage_propagators", "kbe_stage_observables"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libkbe.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_export():
    from paper_2505_19467_amd import kbe
    assert sorted(kbe.EXPORTS) == declared_functions()


def test_workspace_query_sizes():
    from paper_2505_19467_amd import kbe
    for cfg in (inputs.c1(), inputs.c2(), inputs.c4(), inputs.c5()):
        hb, wb, ob = kbe.workspace_query(cfg)
        nk, nb, nt = cfg.nk, cfg.nb, cfg.nt
        # packed, padded lower triangle: at least the packed size, at most ~1% + one row padding more
        packed = nk * 2 * nb * nb * (nt + 1) * (nt + 2) // 2 * 16
        assert packed <= hb <= packed * 1.02 + nk * 2 * nb * nb * 8 * 16 * (nt + 1)
        assert ob == (nt + 1) * 17 * 8
        assert wb > 0
    # C5's history is the ~170 GB of the large workload
    hb, _, _ = kbe.workspace_query(inputs.c5())
    assert 1.6e11 < hb < 1.75e11


def test_workspace_query_rejects_bad_shapes():
    from paper_2505_19467_amd import kbe
    with pytest.raises(kbe.KbeError):
        kbe.workspace_query(inputs.c1().replace(nb=5, hop=inputs.c5().hop))
    with pytest.raises(kbe.KbeError):
        kbe.workspace_query(inputs.c1().replace(nkx=2000))
    with pytest.raises(kbe.KbeError):
        kbe.workspace_query(inputs.c1().replace(dt=-0.1))


def test_row_offsets_are_line_aligned_and_disjoint():
    from paper_2505_19467_amd import kbe
    prev_end = 0
    for j in range(300):
        off = kbe.row_off(j)
        assert off % 8 == 0 and off >= prev_end
        prev_end = off + j + 1
        assert kbe.row_off(j + 1) - off == 8 * ((j + 1 + 7) // 8)
