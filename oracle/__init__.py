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
(their figures are missing from the source).  They are pinned end to end
(Ising closed forms, product states, agreement with the conventional CTMRG,
2x2 cell = 1x1 cell for a translation-invariant state) and network by
network: with no truncation the first projector pairs are resolutions of the
identity, so each teal and red pair of half networks contracts to the plain
norm of the patch it cuts, computed independently from the untouched
environment and site tensors (tests/test_oracle_networks.py; the teal half
networks of App. B likewise, against the column patch closed on itself).
The alternative yellow / red networks of App. B follow complete figures and
are pinned end to end plus exact half-steps (their mirrored yellow pair is
of lower rank and never the identity).
"""
