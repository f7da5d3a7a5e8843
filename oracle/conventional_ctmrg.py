"""Independent conventional double-layer directional CTMRG (numpy, test oracle).

Shares no code with split_ctmrg.  It is the reference the paper compares the
split scheme against (Sec. II A, Fig. CTMRG_Method_2; Sec. III uses
conventional CTMRG with the 2x2-patch projectors of Corboz et al. as the
trusted benchmark).  Ket and bra layers are merged into the double-layer
tensor a = sum_p A A* with D^2-dimensional legs, and every transfer tensor
carries one D^2 leg.

Moves: the left move absorbs one column with projectors built from the full
2x2 patch around each horizontal cut; the other moves are left moves of the
lattice rotated counter-clockwise by 90, 180 and 270 degrees.
"""
from __future__ import annotations

import numpy as np


def _double(A):
    D = A.shape[1]
    a = np.einsum("puldr,pULDR->uUlLdDrR", A, A.conj(), optimize=True)
    return a.reshape(D * D, D * D, D * D, D * D)


def _rot_ccw(env, A, Lx, Ly):
    """Rotate the cell counter-clockwise by 90 degrees: the top edge becomes
    the left edge.  Site [x,y] goes to [-y mod Ly, x]; A'[p,u,l,d,r] =
    A[p,l',...] with u' = r, l' = u, d' = l, r' = d; corners and transfer
    tensors move one position along the ring with their leg order kept."""
    env2, A2 = {}, {}
    for (x, y), e in env.items():
        key = ((-y) % Ly, x)
        env2[key] = dict(C1=e["C2"], C2=e["C3"], C3=e["C4"], C4=e["C1"],
                         T1=e["T2"], T2=e["T3"], T3=e["T4"], T4=e["T1"])
        A2[key] = np.transpose(A[(x, y)], (0, 4, 1, 2, 3))
    return env2, A2, Ly, Lx


def _rotate_k(env, A, Lx, Ly, k):
    for _ in range(k % 4):
        env, A, Lx, Ly = _rot_ccw(env, A, Lx, Ly)
    return env, A, Lx, Ly


def _proj(rT, rB, chi, cutoff):
    """Projectors from two half networks given as matrices [a, b]."""
    M = rB.T @ rT
    U, S, Vh = np.linalg.svd(M)
    if not S[0] > 0:
        raise FloatingPointError("rank-zero projector matrix")
    k = min(chi, int(np.sum(S > cutoff * S[0])))
    w = 1.0 / np.sqrt(S[:k])
    PT = (rB @ U[:, :k]) * w
    PB = (rT @ Vh[:k].T) * w
    return PT, PB


def _left_move(env, A, Lx, Ly, chi, cutoff):
    a = {k: _double(v) for k, v in A.items()}
    for y in range(Ly):
        yn = (y + 1) % Ly
        P = {}
        for x in range(Lx):
            xp = (x + 1) % Lx
            e1, e2, e3, e4 = env[(x, y)], env[(x, yn)], env[(xp, yn)], env[(xp, y)]
            # quadrants of the 2x2 patch: upper-left, upper-right, lower-right, lower-left
            q1 = np.einsum("ab,bce,fga,cghi->fhei", e1["C1"], e1["T1"], e1["T4"], a[(x, y)],
                           optimize=True)             # [T4.d, a.d | T1.r, a.r]
            q2 = np.einsum("ecb,bm,mno,clhn->elho", e2["T1"], e2["C2"], e2["T2"], a[(x, yn)],
                           optimize=True)             # [T1.l, a.l | a.d, T2.d]
            q3 = np.einsum("onm,mt,tli,hrln->hoir", e3["T2"], e3["C3"], e3["T3"], a[(xp, yn)],
                           optimize=True)             # [a.u, T2.u | T3.l, a.l]
            q4 = np.einsum("fgu,tf,qrt,cgri->uciq", e4["T4"], e4["C4"], e4["T3"], a[(xp, y)],
                           optimize=True)             # [T4.u, a.u | a.r, T3.r]
            rT = np.einsum("fhei,eiko->fhko", q1, q2, optimize=True)
            rB = np.einsum("fhcq,koqc->fhko", q4, q3, optimize=True)
            n1, n2 = rT.shape[0] * rT.shape[1], rT.shape[2] * rT.shape[3]
            PT, PB = _proj(rT.reshape(n1, n2), rB.reshape(n1, rB.shape[2] * rB.shape[3]),
                           chi, cutoff)
            P[x] = (PT.reshape(rT.shape[0], rT.shape[1], -1),
                    PB.reshape(rT.shape[0], rT.shape[1], -1))
        new = {}
        for x in range(Lx):
            e = env[(x, y)]
            PT_up, PB_up = P[(x - 1) % Lx]
            PT_dn, _ = P[x]
            _, PB_dn = P[x]
            C1 = np.einsum("ab,bce,ack->ke", e["C1"], e["T1"], PT_up, optimize=True)
            T4 = np.einsum("fga,cghi,ack,fhm->mik", e["T4"], a[(x, y)], PB_up, PT_dn, optimize=True)
            C4 = np.einsum("tv,qrt,vrk->qk", e["C4"], e["T3"], PB_dn, optimize=True)
            new[x] = dict(C1=C1 / np.linalg.norm(C1), T4=T4 / np.linalg.norm(T4),
                          C4=C4 / np.linalg.norm(C4))
        for x in range(Lx):
            site = dict(env[(x, yn)])
            site.update(new[x])
            env[(x, yn)] = site
    return env


def init_identity(Lx, Ly, D):
    """chi = 1 boundary with the ket and bra legs of every edge traced."""
    one = np.ones((1, 1))
    t = np.eye(D).reshape(1, D * D, 1)
    return {(x, y): dict(C1=one, C2=one, C3=one, C4=one, T1=t, T2=t, T3=t, T4=t)
            for x in range(Lx) for y in range(Ly)}


def sweep(env, A, Lx, Ly, chi, cutoff=1e-12):
    """Left, top, right, bottom move."""
    for k in range(4):
        e2, a2, lx, ly = _rotate_k(env, A, Lx, Ly, k)
        e2 = _left_move(e2, a2, lx, ly, chi, cutoff)
        env, _, _, _ = _rotate_k(e2, a2, lx, ly, 4 - k)
    return env


def _vertical_rdm(env, A, x, y, Lx):
    """rho[P,Q,P',Q'] of sites [x,y] (upper, P) and [x+1,y] (lower, Q)."""
    xp = (x + 1) % Lx
    e, f = env[(x, y)], env[(xp, y)]
    A1, A2 = A[(x, y)], A[(xp, y)]
    D = A1.shape[1]

    def split(T):
        return T.reshape(T.shape[0], D, D, T.shape[2])

    top = np.einsum("ab,bcCe,em,mnNo,fgGa,Pcghn,RCGHN->fhHoPR",
                    e["C1"], split(e["T1"]), e["C2"], split(e["T2"]), split(e["T4"]), A1, A1.conj(),
                    optimize=True)
    bot = np.einsum("xgGE,yx,zrRy,wz,FnNw,QKgrn,SLGRN->EKLFQS",
                    split(f["T4"]), f["C4"], split(f["T3"]), f["C3"], split(f["T2"]), A2, A2.conj(),
                    optimize=True)
    return np.einsum("fhHoPR,fhHoQS->PQRS", top, bot, optimize=True)


def _bond(rho, h, swap=False):
    p = rho.shape[0]
    h4 = np.asarray(h).reshape(p, p, p, p)
    if swap:
        h4 = h4.transpose(1, 0, 3, 2)
    num = np.einsum("PQRS,RSPQ->", rho, h4)
    den = np.einsum("PQPQ->", rho)
    return num / den


def energy(env, A, Lx, Ly, h):
    """Energy per site from the vertical bonds of the lattice and of the lattice
    rotated by 90 degrees (whose vertical bonds are the horizontal ones, with
    the right site on top)."""
    tot = 0.0
    for x in range(Lx):
        for y in range(Ly):
            tot += _bond(_vertical_rdm(env, A, x, y, Lx), h)
    e2, a2, lx, ly = _rotate_k(env, A, Lx, Ly, 1)
    for x in range(lx):
        for y in range(ly):
            tot += _bond(_vertical_rdm(e2, a2, x, y, lx), h, swap=True)
    return tot / (Lx * Ly)


def run(A_cell, chi, n_sweeps, cutoff=1e-12):
    """A_cell: array [Lx, Ly, p, D, D, D, D].  Returns the environment."""
    Lx, Ly = A_cell.shape[:2]
    A = {(x, y): np.asarray(A_cell[x, y]) for x in range(Lx) for y in range(Ly)}
    env = init_identity(Lx, Ly, A_cell.shape[3])
    for _ in range(n_sweeps):
        env = sweep(env, A, Lx, Ly, chi, cutoff)
    return env, A
