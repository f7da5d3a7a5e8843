"""Energy as a function of the PEPS tensors, its autograd gradient, and central
finite differences (test oracle).

E(A) is defined as: start from a fixed environment (independent of A), run
exactly n split-CTMRG sweeps (no early stop), evaluate the energy per site.
The gradient is reverse mode through every step including the projector SVDs
(Sec. III: the gradient of the energy by reverse-mode AD through the CTMRG),
using the broadened SVD rule of svd_adjoint.  Truncation ranks are fixed by
the forward pass.

Pinned by central finite differences at D = 2, chi = 4 and at D = 4,
chi = 32, where the kept spectra reach far below 1e-6 s_1 (the broadening of
the SVD adjoint acts per pair of singular values, see svd_adjoint).
"""
from __future__ import annotations

import numpy as np
import torch

from . import split_ctmrg as sc


def energy_of(A_cell: torch.Tensor, env0: dict, chi_E: int, chi_I: int, n_sweeps: int,
              h: np.ndarray, cutoff: float = 1e-12, adj_eps: float = 1e-12, h_v=None,
              alt_yr: bool = False, half_teal: bool = False) -> torch.Tensor:
    """A_cell: [Lx, Ly, p, D, D, D, D] float64 tensor (may require grad);
    h on horizontal bonds, h_v (default h) on vertical ones; alt_yr and
    half_teal select the alternative yellow / red projectors and the teal
    half projectors of App. B."""
    Lx, Ly = A_cell.shape[:2]
    A = {(x, y): A_cell[x, y] for x in range(Lx) for y in range(Ly)}
    env = {k: dict(v) for k, v in env0.items()}
    for _ in range(n_sweeps):
        env = sc.sweep(env, A, Lx, Ly, chi_E, chi_I, cutoff, adj_eps, alt_yr=alt_yr, half_teal=half_teal)
    e, _ = sc.energy(env, A, Lx, Ly, h, h_v)
    return e


def energy_and_grad(A_np: np.ndarray, env0_np: dict, chi_E: int, chi_I: int, n_sweeps: int,
                    h: np.ndarray, cutoff: float = 1e-12, adj_eps: float = 1e-12, h_v=None,
                    alt_yr: bool = False, half_teal: bool = False):
    A = torch.tensor(A_np, dtype=torch.float64, requires_grad=True)
    env0 = sc.env_from_numpy(env0_np)
    e = energy_of(A, env0, chi_E, chi_I, n_sweeps, h, cutoff, adj_eps, h_v, alt_yr, half_teal)
    e.backward()
    return float(e), A.grad.detach().numpy().copy()


def energy_value(A_np, env0_np, chi_E, chi_I, n_sweeps, h, cutoff=1e-12, alt_yr=False,
                 half_teal=False) -> float:
    with torch.no_grad():
        A = torch.tensor(A_np, dtype=torch.float64)
        return float(energy_of(A, sc.env_from_numpy(env0_np), chi_E, chi_I, n_sweeps, h, cutoff,
                               alt_yr=alt_yr, half_teal=half_teal))


def central_difference(A_np, env0_np, chi_E, chi_I, n_sweeps, h, direction, step=1e-4):
    """(E(A + step d) - E(A - step d)) / (2 step)."""
    ep = energy_value(A_np + step * direction, env0_np, chi_E, chi_I, n_sweeps, h)
    em = energy_value(A_np - step * direction, env0_np, chi_E, chi_I, n_sweeps, h)
    return (ep - em) / (2 * step)


def central_difference4(A_np, env0_np, chi_E, chi_I, n_sweeps, h, direction, step=1e-5, alt_yr=False,
                        half_teal=False):
    """Fourth-order central difference
    (8 (E(+s) - E(-s)) - (E(+2s) - E(-2s))) / (12 s)."""
    f = lambda t: energy_value(A_np + t * direction, env0_np, chi_E, chi_I, n_sweeps, h, alt_yr=alt_yr,
                               half_teal=half_teal)
    return (8.0 * (f(step) - f(-step)) - (f(2 * step) - f(-2 * step))) / (12.0 * step)
