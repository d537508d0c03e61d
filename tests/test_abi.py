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
        # packed lower triangle plus at most one unused 64x64 triangle per 64-column strip
        packed = nk * 2 * nb * nb * (nt + 1) * (nt + 2) // 2 * 16
        strips = (nt + 64) // 64
        assert packed <= hb <= packed + nk * 2 * nb * nb * strips * 2016 * 16
        assert ob == (nt + 1) * 17 * 8
        assert wb > 0
    # the large nb = 4 workload's history is ~170 GB (175 GB with the strip padding)
    hb, _, _ = kbe.workspace_query(inputs.c5())
    assert 1.6e11 < hb < 1.8e11


def test_workspace_query_rejects_bad_shapes():
    from paper_2505_19467_amd import kbe
    with pytest.raises(kbe.KbeError):
        kbe.workspace_query(inputs.c1().replace(nb=5, hop=inputs.c5().hop))
    with pytest.raises(kbe.KbeError):
        kbe.workspace_query(inputs.c1().replace(nkx=2000))
    with pytest.raises(kbe.KbeError):
        kbe.workspace_query(inputs.c1().replace(dt=-0.1))


def test_history_layout_is_a_bijection():
    """Every stored (c, t_j, t') of one k maps to a distinct offset inside its C * P elements;
    each row segment of a strip holds the C components' 64-element segments back to back, and
    consecutive rows of a strip follow each other (one contiguous stream per strip)."""
    import numpy as np
    from paper_2505_19467_amd import kbe
    for fp32 in (False, True):
        for nt, C in ((1, 2), (63, 8), (64, 8), (65, 2), (200, 8), (1000, 8), (130, 32), (70, 18)):
            P = kbe.plane_length(nt)
            j, tp = np.tril_indices(nt + 1)
            c = np.repeat(np.arange(C), len(j))
            off = kbe.hist_offset(c, np.tile(j, C), np.tile(tp, C), nt, C, fp32)
            assert off.min() >= 0 and off.max() < C * P
            assert len(np.unique(off)) == len(off)
            # fill factor: the unused part is at most one 64x64 triangle per strip and component
            assert C * P - len(off) <= C * ((nt + 64) // 64) * 64 * 63 // 2
            for s in range(0, (nt + 1 + 63) // 64):
                rows = np.arange(64 * s, nt + 1)
                first = kbe.hist_offset(0, rows, np.full_like(rows, 64 * s), nt, C, fp32)
                assert np.all(np.diff(first) == 64 * C)
                last = kbe.hist_offset(C - 1, rows, np.full_like(rows, 64 * s + 63), nt, C, fp32)
                assert np.all(last - first == 64 * C - 1)
            if fp32:  # a column's component pair is adjacent: one 16-byte load
                pair = kbe.hist_offset(np.array([0, 1]), 64, 5, nt if nt >= 64 else 64, C, True)
                assert pair[1] - pair[0] == 1


def test_mfma_history_layout_is_a_bijection():
    """FP32-MFMA quad layout: every stored (c, t_j, t') of one k maps to a distinct offset inside
    its C * P elements; a quad of 4 rows of a strip is one contiguous run of 256 C elements and
    the quads of a strip follow each other; for one (quad, column group, component pair) the 64
    lanes L = 16 (j % 4) + (t' % 16) read 64 consecutive 16-byte pairs (one 1 KB load)."""
    import numpy as np
    from paper_2505_19467_amd import kbe
    for nt, C in ((1, 2), (63, 8), (64, 8), (65, 2), (200, 8), (1000, 8), (130, 32), (70, 18), (66, 32)):
        N = nt + 1
        P = kbe.plane_length(nt, mfma=True)
        j, tp = np.tril_indices(N)
        c = np.repeat(np.arange(C), len(j))
        off = kbe.hist_offset(c, np.tile(j, C), np.tile(tp, C), nt, C, True, True)
        assert off.min() >= 0 and off.max() < C * P
        assert len(np.unique(off)) == len(off)
        # unused: one 64x64 triangle per strip and component, plus at most 3 padding rows per strip
        assert C * P - len(off) <= C * ((nt + 64) // 64) * (64 * 63 // 2 + 3 * 64)
        for s in range(0, (N + 63) // 64):
            nq = (N - 64 * s + 3) // 4
            assert kbe.quad_base(s + 1, N) - kbe.quad_base(s, N) == nq
            rows = np.arange(64 * s, N)
            starts = kbe.hist_offset(0, rows[::4], np.full(len(rows[::4]), 64 * s), nt, C, True, True)
            assert np.all(np.diff(starts) == 256 * C)
        # one 16-byte load of lane L: components 2 ci, 2 ci + 1 of its pair are adjacent, and
        # lane L + 1 continues where lane L ends
        s, q, g, ci = 0, 8, 1, C // 2 - 1   # rows 32..35, columns 16..31: all stored
        lanes = np.arange(64)
        jj, tt = 64 * s + 4 * q + lanes // 16, 64 * s + 16 * g + lanes % 16
        keep = tt <= jj
        assert keep.all()
        e0 = kbe.hist_offset(2 * ci, jj, tt, max(nt, 80), C, True, True)
        e1 = kbe.hist_offset(2 * ci + 1, jj, tt, max(nt, 80), C, True, True)
        assert np.all(e1 - e0 == 1)
        assert np.all(e0[keep] == e0[0] + 2 * lanes[keep])


def test_create_rejects_undersized_buffers():
    """kbe_create checks every buffer size against the layout of its own config before it
    launches anything (so this runs without a GPU): one element short in any buffer, or a
    workspace sized for a shorter run, is refused."""
    from paper_2505_19467_amd import kbe
    import numpy as np
    cfg = inputs.c1()
    c = kbe._c_config(cfg, 20)
    hb, wb, ob = kbe._query(c)
    _, wb_short, _ = kbe._query(kbe._c_config(cfg, 10))
    assert wb_short < wb
    hop = np.ascontiguousarray(cfg.hop, np.complex128).view(np.float64)
    fake = ctypes.c_void_p(0x100000)  # never dereferenced: the size check comes first
    ctx = ctypes.c_void_p()
    dp = hop.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    for sizes in ((hb, wb_short, ob), (hb - 16, wb, ob), (hb, wb - 256, ob), (hb, wb, ob - 8)):
        rc = kbe._lib.kbe_create(ctypes.byref(c), dp, None, fake, sizes[0], fake, sizes[1], fake, sizes[2],
                                 None, ctypes.byref(ctx))
        assert rc == -1 and not ctx.value


def test_adjoint_query():
    from paper_2505_19467_amd import kbe
    n = ctypes.c_size_t()
    cfg = inputs.c4()
    hb, _, _ = kbe.workspace_query(cfg)
    assert kbe._lib.kbe_adjoint_query(ctypes.byref(kbe._c_config(cfg, None)), ctypes.byref(n)) == 0
    assert n.value > hb  # the adjoint history alone has the FP64 history's size
    # K = 2, the FP32 form and nb > 2 are outside the reverse sweep
    for bad in (cfg.replace(n_corr=2), cfg.replace(precision=inputs.PRECISION_FP32), inputs.c5()):
        assert kbe._lib.kbe_adjoint_query(ctypes.byref(kbe._c_config(bad, None)), ctypes.byref(n)) == -2


def test_corrector_tolerance_sizes_and_errors():
    """corr_tol > 0 adds the per-(k, t') change buffer (and its maximum) to the workspace;
    negative or non-finite tolerances, and a tolerance without corrector passes, are refused;
    the adjoint needs the fixed-count corrector."""
    from paper_2505_19467_amd import kbe
    cfg = inputs.c2()
    _, w0, _ = kbe.workspace_query(cfg)
    _, w1, _ = kbe.workspace_query(cfg.replace(n_corr=4, corr_tol=1e-8))
    need = cfg.nk * (((cfg.nt + 1 + 7) // 8) * 8) * 8
    assert need <= w1 - w0 <= need + 1024
    for bad in (cfg.replace(corr_tol=-1.0), cfg.replace(corr_tol=float("nan")), cfg.replace(corr_tol=float("inf")),
                cfg.replace(n_corr=0, corr_tol=1e-8)):
        with pytest.raises(kbe.KbeError):
            kbe.workspace_query(bad)
    n = ctypes.c_size_t()
    tol = inputs.c4().replace(n_corr=1, corr_tol=1e-8)
    assert kbe._lib.kbe_adjoint_query(ctypes.byref(kbe._c_config(tol, None)), ctypes.byref(n)) == -2
    assert kbe._lib.kbe_corrector_log(None, 0, 1, None, None) == -1


def test_interband_chain_and_pulse_validation():
    """The interband preset needs nb = 2 and adds the real-space lines of the current row to the
    workspace; chains of up to 1024 points are accepted, 2D grids up to 64 per axis; an unknown
    pulse kind, or a dipole kick with nb != 2 or t0 < 0, is refused before anything touches the
    device; the adjoint refuses the interband preset and chains longer than 64."""
    from paper_2505_19467_amd import kbe
    import numpy as np
    p1 = inputs.paper_chain()
    _, wb, _ = kbe.workspace_query(p1)
    _, wb_h, _ = kbe.workspace_query(p1.replace(interaction=inputs.INTERACTION_HUBBARD))
    Tp = ((p1.nt + 1 + 7) // 8) * 8
    need = Tp * 8 * p1.nk * 16
    assert need <= wb - wb_h <= need + 1024
    for bad in (p1.replace(nkx=1025), inputs.c2().replace(nkx=65), inputs.c2().replace(nkx=40, nky=40),
                inputs.c5().replace(interaction=inputs.INTERACTION_INTERBAND)):
        with pytest.raises(kbe.KbeError):
            kbe.workspace_query(bad)
    n = ctypes.c_size_t()
    for bad in (p1.replace(nkx=16, pulse=inputs.Pulse()), inputs.c1().replace(nkx=128)):
        assert kbe._lib.kbe_adjoint_query(ctypes.byref(kbe._c_config(bad, None)), ctypes.byref(n)) == -2
    assert kbe._lib.kbe_adjoint_query(ctypes.byref(kbe._c_config(inputs.c1().replace(nkx=64), None)),
                                      ctypes.byref(n)) == 0
    # pulse checks come before any buffer is used: fake device pointers are never dereferenced
    fake = ctypes.c_void_p(0x100000)
    for cfg, kind, t0 in ((p1.replace(nkx=16, nt=20), 2, 0.5), (p1.replace(nkx=16, nt=20), 1, -0.1),
                          (inputs.c5().replace(nkx=2, nky=2, nt=8), 1, 0.5)):
        c = kbe._c_config(cfg, None)
        hb, wb, ob = kbe._query(c)
        hop = np.ascontiguousarray(cfg.hop, np.complex128).view(np.float64)
        pu = kbe.KbePulse(amp=0.3, omega=0.0, t0=t0, width=1.0, pol=(ctypes.c_double * 2)(1.0, 0.0), kind=kind)
        ctx = ctypes.c_void_p()
        rc = kbe._lib.kbe_create(ctypes.byref(c), hop.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 ctypes.byref(pu), fake, hb, fake, wb, fake, ob, None, ctypes.byref(ctx))
        assert rc == -1 and not ctx.value


def _header_enums():
    """name -> value of every enumerator in include/kbe.h."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for body in re.findall(r"enum\s*\{(.*?)\}", text, flags=re.S):
        for name, value in re.findall(r"\b(KBE_[A-Z0-9_]+)\s*=\s*(-?\d+)", body):
            out[name] = int(value)
    return out


def _header_struct_fields(typedef):
    """[(c type, field name)] of a typedef'd struct in include/kbe.h, in declaration order."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct\s*\{([^{}]*)\}\s*" + typedef + r"\s*;", text, flags=re.S).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        ctype, names = decl.split(None, 1)
        for n in names.split(","):
            fields.append((ctype, n.strip()))
    return fields


def test_binding_constants_match_header():
    from paper_2505_19467_amd import kbe
    e = _header_enums()
    assert kbe.KBE_OK == e["KBE_OK"]
    assert {v: k for k, v in kbe.ERRORS.items()} == {k: v for k, v in e.items() if k.startswith("KBE_ERR_")}
    assert kbe.NOBS == e["KBE_NOBS"]
    for col, name in [("t", "KBE_OBS_T"), ("N", "KBE_OBS_N"), ("Ekin", "KBE_OBS_EKIN"), ("EHF", "KBE_OBS_EHF"),
                      ("Ecorr", "KBE_OBS_ECORR"), ("Etot", "KBE_OBS_ETOT"), ("Jx", "KBE_OBS_JX"), ("Jy", "KBE_OBS_JY"),
                      ("A", "KBE_OBS_A"), ("n_orb0", "KBE_OBS_NORB"), ("n_band0", "KBE_OBS_NBAND")]:
        assert kbe.OBS[col] == e[name], col
    for n in ("SIGMA", "I_PREV", "I_CUR", "RHO_PREV", "RHO_CUR", "D_PREV", "D_CUR", "PROP", "COL0", "DIAG", "ROWS"):
        assert getattr(kbe, "BUF_" + n) == e["KBE_BUF_" + n], n
    assert (inputs.PRECISION_FP64, inputs.PRECISION_FP32, inputs.PRECISION_FP32_MFMA) == \
        (e["KBE_FP64"], e["KBE_FP32"], e["KBE_FP32_MFMA"])
    mx = re.search(r"#define KBE_NOALLOC_WORKSPACE_MAX \(\(size_t\)(\d+) << (\d+)\)", open(HEADER).read())
    assert kbe.NOALLOC_WORKSPACE_MAX == int(mx.group(1)) << int(mx.group(2))
    assert (inputs.INTERACTION_HUBBARD, inputs.INTERACTION_INTERBAND) == (e["KBE_INT_HUBBARD"], e["KBE_INT_INTERBAND"])
    assert (inputs.PULSE_PEIERLS, inputs.PULSE_DIPOLE_KICK) == (e["KBE_PULSE_PEIERLS"], e["KBE_PULSE_DIPOLE_KICK"])


@pytest.mark.parametrize("typedef,cls", [("kbe_config", "KbeConfig"), ("kbe_pulse", "KbePulse")])
def test_binding_structs_match_header(typedef, cls):
    """Field names, order and C types of the ctypes mirrors equal the header's structs."""
    from paper_2505_19467_amd import kbe
    ctypes_of = {"int32_t": ctypes.c_int32, "double": ctypes.c_double}
    want = []
    for ctype, name in _header_struct_fields(typedef):
        m = re.fullmatch(r"(\w+)\[(\d+)\]", name)
        want.append((m.group(1), ctypes_of[ctype] * int(m.group(2))) if m else (name, ctypes_of[ctype]))
    got = getattr(kbe, cls)._fields_
    assert [n for n, _ in got] == [n for n, _ in want]
    for (n, t), (_, w) in zip(got, want):
        assert ctypes.sizeof(t) == ctypes.sizeof(w) and getattr(t, "_type_", t) == getattr(w, "_type_", w), n
