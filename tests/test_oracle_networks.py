"""Network-level pins of the oracle's teal and red half networks (CPU).

The teal and red networks are a reading of the paper (their figure bodies are
missing), so no printed value pins them one by one.  What the mathematics
fixes is this: the first projector pairs (green, yellow and their mirrored
primes) are resolutions of the identity when nothing is truncated (a pair
P_T, P_B built from half networks of full row rank with every singular value
kept satisfies P_B P_T^T = 1 on the truncated legs), so contracting the upper
and lower half networks of a cut with each other must give the plain norm of
the patch they cut, contracted here from the untouched environment tensors
and site tensors with numpy's einsum (no oracle code):

  teal: sum rho^T rho^B = the 2 x 2 patch of rows x, x+1 and columns y, y+1;
  red:  sum rho^T rho^B = the 1 x 2 patch of row x;
  teal half networks (App. B): the 2 x 1 patch of column y with its right
        side closed on itself (top-edge bond to bottom-edge bond, each
        layer's right leg of row x to that of row x+1).

A wrong leg, a tensor from the wrong site or a missing one in any of these
networks changes the scalar for random tensors.  App. A first projectors
(with the App. A and the App. B teal networks), 1x1 and 2x2 cells.  The
App. B alternative yellow / red construction is not covered: its mirrored
yellow' pair cuts (p, D, chi_I) legs against a half network of dimension
chi_I D, so it is an oblique projector of lower rank, never the identity
(those networks follow complete figures and are pinned by their exact
half-steps in test_oracle.py).
"""
import os
import string
import sys

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import split_ctmrg as sc  # noqa: E402
from paper_2502_10298_amd import inputs as inp  # noqa: E402

D, P, CHI_E, CHI_I = 2, 2, 4, 2       # every first half network has full row rank
KEEP = 16                             # new bond dimensions large enough that nothing is truncated


def contract(terms, out=()):
    """Contraction of [(array, [bond names])]: every name not in `out` sits on
    exactly two legs and is summed; the result has the legs `out` (a float
    when `out` is empty)."""
    names = sorted({n for _, legs in terms for n in legs} | set(out))
    letters = dict(zip(names, string.ascii_letters))
    assert len(names) <= len(string.ascii_letters)
    for n in names:
        assert sum(legs.count(n) for _, legs in terms) == (1 if n in out else 2), n
    spec = ",".join("".join(letters[n] for n in legs) for _, legs in terms) + "->" + "".join(letters[n] for n in out)
    r = np.einsum(spec, *[t for t, _ in terms], optimize="greedy")
    return float(r) if not out else r


def patch_1x2(eL, eR, aL, aR):
    """Row patch: left site (environment eL, tensor aL) and right site (eR, aR)."""
    return contract([
        (eL["C1"], ["l3", "t1"]), (eL["T1k"], ["t1", "kLu", "t2"]), (eL["T1b"], ["t2", "bLu", "t3"]),
        (eR["T1k"], ["t3", "kRu", "t4"]), (eR["T1b"], ["t4", "bRu", "t5"]), (eR["C2"], ["t5", "r1"]),
        (eR["T2k"], ["r1", "kRr", "r2"]), (eR["T2b"], ["r2", "bRr", "r3"]), (eR["C3"], ["r3", "o1"]),
        (eR["T3b"], ["o1", "bRd", "o2"]), (eR["T3k"], ["o2", "kRd", "o3"]), (eL["T3b"], ["o3", "bLd", "o4"]),
        (eL["T3k"], ["o4", "kLd", "o5"]), (eL["C4"], ["o5", "l1"]), (eL["T4b"], ["l1", "bLl", "l2"]),
        (eL["T4k"], ["l2", "kLl", "l3"]),
        (aL, ["pL", "kLu", "kLl", "kLd", "kh"]), (aL, ["pL", "bLu", "bLl", "bLd", "bh"]),
        (aR, ["pR", "kRu", "kh", "kRd", "kRr"]), (aR, ["pR", "bRu", "bh", "bRd", "bRr"]),
    ])


def patch_2x2(eTL, eTR, eBL, eBR, aTL, aTR, aBL, aBR):
    """2 x 2 patch: top row (TL, TR) over bottom row (BL, BR), contracted as
    four corner blocks (each corner's environment and its site in both
    layers), then the two rows, then the rows with each other."""
    TL = contract([(eTL["C1"], ["l5", "t1"]), (eTL["T1k"], ["t1", "kTLu", "t2"]), (eTL["T1b"], ["t2", "bTLu", "t3"]),
                   (eTL["T4b"], ["l3", "bTLl", "l4"]), (eTL["T4k"], ["l4", "kTLl", "l5"]),
                   (aTL, ["pTL", "kTLu", "kTLl", "kTLd", "kTh"]), (aTL, ["pTL", "bTLu", "bTLl", "bTLd", "bTh"])],
                  out=["t3", "l3", "kTLd", "bTLd", "kTh", "bTh"])
    TR = contract([(eTR["T1k"], ["t3", "kTRu", "t4"]), (eTR["T1b"], ["t4", "bTRu", "t5"]), (eTR["C2"], ["t5", "r1"]),
                   (eTR["T2k"], ["r1", "kTRr", "r2"]), (eTR["T2b"], ["r2", "bTRr", "r3"]),
                   (aTR, ["pTR", "kTRu", "kTh", "kTRd", "kTRr"]), (aTR, ["pTR", "bTRu", "bTh", "bTRd", "bTRr"])],
                  out=["t3", "r3", "kTRd", "bTRd", "kTh", "bTh"])
    BR = contract([(eBR["T2k"], ["r3", "kBRr", "r4"]), (eBR["T2b"], ["r4", "bBRr", "r5"]), (eBR["C3"], ["r5", "o1"]),
                   (eBR["T3b"], ["o1", "bBRd", "o2"]), (eBR["T3k"], ["o2", "kBRd", "o3"]),
                   (aBR, ["pBR", "kTRd", "kBh", "kBRd", "kBRr"]), (aBR, ["pBR", "bTRd", "bBh", "bBRd", "bBRr"])],
                  out=["r3", "o3", "kTRd", "bTRd", "kBh", "bBh"])
    BL = contract([(eBL["T3b"], ["o3", "bBLd", "o4"]), (eBL["T3k"], ["o4", "kBLd", "o5"]), (eBL["C4"], ["o5", "l1"]),
                   (eBL["T4b"], ["l1", "bBLl", "l2"]), (eBL["T4k"], ["l2", "kBLl", "l3"]),
                   (aBL, ["pBL", "kTLd", "kBLl", "kBLd", "kBh"]), (aBL, ["pBL", "bTLd", "bBLl", "bBLd", "bBh"])],
                  out=["o3", "l3", "kTLd", "bTLd", "kBh", "bBh"])
    top = contract([(TL, ["t3", "l3", "kTLd", "bTLd", "kTh", "bTh"]), (TR, ["t3", "r3", "kTRd", "bTRd", "kTh", "bTh"])],
                   out=["l3", "kTLd", "bTLd", "r3", "kTRd", "bTRd"])
    bottom = contract([(BL, ["o3", "l3", "kTLd", "bTLd", "kBh", "bBh"]),
                       (BR, ["r3", "o3", "kTRd", "bTRd", "kBh", "bBh"])],
                      out=["l3", "kTLd", "bTLd", "r3", "kTRd", "bTRd"])
    return float((top * bottom).sum())


def patch_2x1_closed(eT, eB, aT, aB):
    """Column patch (top site eT, aT over bottom site eB, aB) whose right side
    is closed on itself: the top edge's bond to the bottom edge's, and each
    layer's right leg of the top site to that of the bottom site."""
    return contract([
        (eT["C1"], ["l5", "t1"]), (eT["T1k"], ["t1", "kTu", "t2"]), (eT["T1b"], ["t2", "bTu", "h"]),
        (eB["T3b"], ["h", "bBd", "o4"]), (eB["T3k"], ["o4", "kBd", "o5"]), (eB["C4"], ["o5", "l1"]),
        (eB["T4b"], ["l1", "bBl", "l2"]), (eB["T4k"], ["l2", "kBl", "l3"]),
        (eT["T4b"], ["l3", "bTl", "l4"]), (eT["T4k"], ["l4", "kTl", "l5"]),
        (aT, ["pT", "kTu", "kTl", "kv", "kr"]), (aT, ["pT", "bTu", "bTl", "bv", "br"]),
        (aB, ["pB", "kv", "kBl", "kBd", "kr"]), (aB, ["pB", "bv", "bBl", "bBd", "br"]),
    ])


def networks(env, A, Lx, Ly, y, x, alt_yr, half_teal):
    yn = (y + 1) % Ly
    G, Y, Gr, Yr = sc._first_projectors(env, A, Lx, y, KEEP, KEEP, 1e-12, 1e-12, alt_yr)
    if yn != y:
        Gr, Yr = sc._first_projectors(env, A, Lx, yn, KEEP, KEEP, 1e-12, 1e-12, alt_yr)[2:]
    for pr in list(G.values()) + list(Y.values()) + list(Gr.values()) + list(Yr.values()):
        PT, PB, S, k = pr
        assert k == PT.shape[-1] and k == int(np.prod(PT.shape[:-1])), "a projector truncates"
    left = sc.left_intermediate(env, A, Lx, y, G, Y, alt_yr)
    right = sc.right_intermediate(env, A, Lx, yn, Gr, Yr, alt_yr)
    return sc.teal_red_networks(env, A, Lx, y, yn, x, left, right, alt_yr, half_teal)


@pytest.mark.parametrize("Lx,Ly", [(1, 1), (2, 2)])
@pytest.mark.parametrize("half_teal", [False, True])
def test_teal_and_red_networks_close_to_the_patch_norms(Lx, Ly, half_teal):
    alt_yr = False
    env_np = inp.random_env(71 + Lx, Lx, Ly, D, CHI_E, CHI_I)
    A_np = inp.peps_gaussian(72 + Lx, Lx, Ly, P, D)
    env = sc.env_from_numpy(env_np)
    A = sc.peps_from_numpy(A_np)
    a = {k: A_np[k[0], k[1]] for k in env_np}
    with torch.no_grad():
        for x in range(Lx):
            for y in range(Ly):
                xp, yn = (x + 1) % Lx, (y + 1) % Ly
                rT, rB, sT, sB, _ = networks(env, A, Lx, Ly, y, x, alt_yr, half_teal)
                teal = float((rT * rB).sum())
                red = float((sT * sB).sum())
                if half_teal:
                    ref_teal = patch_2x1_closed(env_np[(x, y)], env_np[(xp, y)], a[(x, y)], a[(xp, y)])
                else:
                    ref_teal = patch_2x2(env_np[(x, y)], env_np[(x, yn)], env_np[(xp, y)], env_np[(xp, yn)],
                                         a[(x, y)], a[(x, yn)], a[(xp, y)], a[(xp, yn)])
                ref_red = patch_1x2(env_np[(x, y)], env_np[(x, yn)], a[(x, y)], a[(x, yn)])
                # rounding only: the projector pairs carry s^(-1/2) of half
                # networks with condition numbers up to ~1e5 here
                assert abs(teal - ref_teal) <= 1e-8 * abs(ref_teal), (x, y, teal, ref_teal)
                assert abs(red - ref_red) <= 1e-8 * abs(ref_red), (x, y, red, ref_red)
