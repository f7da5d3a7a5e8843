"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every symbol the header declares, and its dry-run workspace planner walks the
whole contraction plan (every network's index bookkeeping) for each workload."""
import os
import re

import pytest

from paper_2502_10298_amd import binding as b
from paper_2502_10298_amd import inputs as inp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "splitctm.h")).read()
    return sorted(set(re.findall(r"\b(ctm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = b.lib()
    names = _declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(b.EXPORTED) <= set(names)


def test_strerror_never_null():
    for s in range(-1, 8):
        assert isinstance(b.strerror(s), str) and b.strerror(s)


@pytest.mark.parametrize("name", list(inp.WORKLOADS))
def test_dry_run_workspace_plan(name):
    w = inp.WORKLOADS[name]
    cfg = b.make_config(w["Lx"], w["Ly"], w["p"], w["D"], w["chi"], w["chi"],
                        "fp64" if w["prec"] == "fp64" else "fp32")
    fwd = b.workspace_size(cfg)
    grad = b.workspace_size(cfg, True, w.get("sweeps") or 5, w.get("ckpt", 1))
    assert 0 < fwd <= grad < 200 * 2**30


def test_invalid_configs_rejected():
    bad = [b.make_config(0, 1, 2, 2, 8, 8), b.make_config(1, 1, 2, 4, 8, 2),   # chi_I < D with identity
           b.make_config(1, 1, 2, 2, 0, 8)]
    for cfg in bad:
        with pytest.raises(b.CtmError):
            b.workspace_size(cfg)


def test_debug_decompositions_reject_sizes_beyond_their_limits():
    # the argument checks run before any device call, so the (never
    # dereferenced) pointers may be dummies and no GPU is needed
    import ctypes
    L = b.lib()
    d = ctypes.c_void_p(256)
    sw = ctypes.c_int(0)
    assert L.ctm_debug_svd(4097, 1, d, d, d, d, d, ctypes.byref(sw), None) == b.CTM_EINVAL
    assert L.ctm_debug_svd(0, 1, d, d, d, d, d, ctypes.byref(sw), None) == b.CTM_EINVAL
    assert L.ctm_debug_qr(8193, 16, 1, d, d, d, d, None) == b.CTM_EINVAL
    assert L.ctm_debug_qr(16, 17, 1, d, d, d, d, None) == b.CTM_EINVAL   # k > m


def test_projector_variants_and_svd_limits_validated():
    """Every projector construction plans at the headline size; a teal half
    projector matrix beyond the rank-limited route's 8192 rows (chi_E D^2 at
    chi = 170, D = 8) and an unknown variant flag are rejected up front."""
    for alt, half in ((False, False), (True, False), (False, True), (True, True)):
        cfg = b.make_config(2, 2, 2, 8, 128, 128, "bf16x3", alt_yr=alt, half_teal=half)
        assert b.workspace_size(cfg, True, 4, 4) > 0
    with pytest.raises(b.CtmError):
        b.workspace_size(b.make_config(1, 1, 2, 8, 170, 170, "bf16x3", half_teal=True))
    assert b.workspace_size(b.make_config(1, 1, 4, 12, 170, 170, "bf16x3")) > 0
    cfg = b.make_config(1, 1, 2, 2, 8, 8)
    cfg.projector_variant = 4
    with pytest.raises(b.CtmError):
        b.workspace_size(cfg)
