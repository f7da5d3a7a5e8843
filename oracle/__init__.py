"""Test infrastructure: plain, slow FP64 CPU oracles for the split-CTMRG hot path.

Nothing in the product path imports this package.  Only the tests, the smoke
check and the CPU-baseline leg of the benchmark call it.

Modules
-------
split_ctmrg
    The split-CTMRG method (torch CPU float64): projector recipe, one left
    move with green/yellow then teal/red projectors, the other three moves by
    lattice symmetry, sweeps, the nearest-neighbour energy, Ising free energy
    and magnetisation helpers; the App. B constructions (alternative
    yellow / red projectors with the physical leg cut by yellow, teal half
    projectors) behind the alt_yr / half_teal flags.
svd_adjoint
    Broadened SVD used by the oracle gradient (torch autograd Function).
grad
    E(A) as a differentiable function (fixed sweep count from a fixed start)
    and central finite differences.
conventional_ctmrg
    An independent double-layer directional CTMRG (numpy) with 2x2-patch
    projectors, sharing no code with split_ctmrg.

Parity status: the teal and red half networks are a reading of the paper
(their figures are missing from the source); they are pinned end to end only
(Ising closed forms, product states, agreement with the conventional CTMRG,
2x2 cell = 1x1 cell for a translation-invariant state), not network by
network: "parity unpinned" at the level of the individual teal / red
networks.  The same holds for the teal half networks of App. B (their figure
has no body either): pinned end to end by product states, Onsager and
convergence to the conventional CTMRG.  The alternative yellow / red networks
follow complete figures and are pinned the same way, plus exact half-steps.
"""
