"""Variational optimisation of the PEPS tensors with L-BFGS (Sec. III: the
energy is minimised over the tensors, each step taking the energy and its
gradient from the CTMRG and its reverse pass; Fig. timing_at_otpimization
times such steps).

A thin host loop: torch's L-BFGS over CtmEnergy, every evaluation running
`n_sweeps` split-CTMRG sweeps on the GPU from the environment the previous
evaluation ended with (warm start), then the energy and dE/dA.  The energy is
a function of A alone up to that start environment.
"""
from __future__ import annotations

import time

import torch

from . import binding as b


def lbfgs(A0, h, chi_E, steps, n_sweeps=4, ckpt_every=4, prec="bf16x3", pre_sweeps=8, chi_I=None, h_v=None,
          history_size=10, line_search="strong_wolfe", alt_yr=False, half_teal=False, on_eval=None):
    """Run `steps` L-BFGS iterations from A0 (FP64 device tensor
    [Lx, Ly, p, D, D, D, D]).  The start environment is `pre_sweeps` sweeps
    from the identity boundary at A0.  Returns (A, history) with history a
    list of dicts, one per energy + gradient evaluation: energy, gradient
    norm, wall seconds, L-BFGS iteration."""
    obj = b.SplitCTM(A0.detach(), chi_E, chi_I if chi_I is not None else chi_E, prec=prec, alt_yr=alt_yr,
                     half_teal=half_teal)
    obj.sweep(pre_sweeps)
    state = {"env": obj.env_export()}
    obj.close()
    A = A0.detach().clone().requires_grad_(True)
    opt = torch.optim.LBFGS([A], lr=1.0, max_iter=steps, max_eval=4 * steps, history_size=history_size,
                            tolerance_grad=0.0, tolerance_change=0.0, line_search_fn=line_search)
    history = []

    def closure():
        opt.zero_grad()
        t0 = time.perf_counter()
        e = b.ctm_energy(A, h, chi_E, n_sweeps, ckpt_every, prec, chi_I=chi_I, h_v=h_v, alt_yr=alt_yr,
                         half_teal=half_teal, state=state)
        e.backward()
        torch.cuda.synchronize()
        rec = {"energy": float(e), "grad_norm": float(A.grad.norm()), "seconds": time.perf_counter() - t0,
               "iteration": opt.state[A].get("n_iter", 0)}
        history.append(rec)
        if on_eval is not None:
            on_eval(rec)
        return e

    opt.step(closure)
    return A.detach(), history
