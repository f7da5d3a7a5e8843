"""The allocation-free context (ctm_init_static: the library's static device
array as the workspace) against the context on a caller-owned workspace
(ctm_init), through the C ABI: the same sweeps, energies, environment and
gradient, on two calls in a row, the second with a smaller input."""
import numpy as np
import pytest
import torch

from paper_2502_10298_amd import binding as b
from paper_2502_10298_amd import inputs as inp

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(*a):
    print("[case]", *a, flush=True)


def _run(A_np, chi, static):
    h = inp.heisenberg_h_rotated()
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), chi, prec="fp64", with_grad=True, n_sweeps=2, ckpt_every=1,
                     static_workspace=static)
    st, n, delta = obj.sweep(8)
    e, bonds = obj.energy(h)
    env = obj.env_export()
    eg, dA = obj.energy_grad(h, 2, 1)
    obj.close()
    return e, bonds, env, eg, dA


def test_static_context_matches_workspace_context():
    """Two calls in a row (D = 2, chi = 8, then the smaller D = 2, chi = 5
    with another seed): every output of the static context equals the
    workspace context's to 1e-12 relative (FP64; the two run the same
    kernels on the same inputs, only the workspace address differs)."""
    for seed, chi in ((1234, 8), (77, 5)):
        A_np = inp.peps_gaussian(seed, 1, 1, 2, 2)
        _say(f"static context, D=2 chi={chi}")
        e_s, bonds_s, env_s, eg_s, dA_s = _run(A_np, chi, True)
        _say(f"workspace context, D=2 chi={chi}")
        e_w, bonds_w, env_w, eg_w, dA_w = _run(A_np, chi, False)
        assert abs(e_s - e_w) <= 1e-12 * abs(e_w)
        assert np.allclose(bonds_s, bonds_w, rtol=0, atol=1e-12 * np.abs(bonds_w).max())
        assert torch.allclose(env_s, env_w, rtol=0, atol=1e-12 * float(env_w.abs().max()))
        assert abs(eg_s - eg_w) <= 1e-12 * abs(eg_w)
        assert torch.allclose(dA_s, dA_w, rtol=0, atol=1e-12 * float(dA_w.abs().max()))


def test_static_context_limits():
    """A configuration whose workspace exceeds the static array, and a second
    static context on a device whose array belongs to a live context, are
    CTM_EINVAL; after ctm_destroy the array is free again."""
    A_big = torch.tensor(inp.peps_gaussian(5, 2, 2, 2, 8), device=DEV)
    _say("static context beyond the array")
    with pytest.raises(b.CtmError) as ex:
        b.SplitCTM(A_big, 128, prec="bf16x3", static_workspace=True)
    assert ex.value.status == b.CTM_EINVAL
    A = torch.tensor(inp.peps_gaussian(6, 1, 1, 2, 2), device=DEV)
    first = b.SplitCTM(A, 4, prec="fp64", static_workspace=True)
    _say("second static context while the first is alive")
    with pytest.raises(b.CtmError) as ex:
        b.SplitCTM(A, 4, prec="fp64", static_workspace=True)
    assert ex.value.status == b.CTM_EINVAL
    first.close()
    again = b.SplitCTM(A, 4, prec="fp64", static_workspace=True)
    again.sweep(2)
    again.close()
