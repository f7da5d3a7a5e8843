"""Seeded synthetic inputs shared by the oracle tests, the GPU path and bench.py.

This module holds no arithmetic of the split-CTMRG method: it draws random
PEPS tensors and random environments, builds the fixed test Hamiltonians and
the square-root-Boltzmann Ising PEPS used as a closed-form pin, and packs or
unpacks environments into the flat layout that crosses the C ABI.

Leg conventions (the paper draws the legs but never names them):

    A[p,u,l,d,r]                     physical, up, left, down, right
    C1[d,r] C2[l,d] C3[u,l] C4[r,u]  corners, each ordered (in, out) along the
                                     ring C1 -> T1 -> C2 -> T2 -> C3 -> T3 -> C4 -> T4
    T1k[l,s,r] T1b[l,s,r]            top edge,    C1 -> T1k -> T1b -> C2
    T2k[u,s,d] T2b[u,s,d]            right edge,  C2 -> T2k -> T2b -> C3
    T3b[r,s,l] T3k[r,s,l]            bottom edge, C3 -> T3b -> T3k -> C4
    T4b[d,s,u] T4k[d,s,u]            left edge,   C4 -> T4b -> T4k -> C1

The first tensor along each edge (T1k, T2k, T3b, T4b) has shape [chi_E, D, chi_I]
and the second (T1b, T2b, T3k, T4k) has shape [chi_I, D, chi_E] (split transfer
tensors of Sec. II B, Fig. split-transfer-ctmrg).  Sites are [x, y] with x the
row and y the column; the cell is periodic.
"""
from __future__ import annotations

import numpy as np

# Order in which the twelve tensors of one site are packed (ring order).
ENV_NAMES = ("C1", "C2", "C3", "C4",
             "T1k", "T1b", "T2k", "T2b", "T3b", "T3k", "T4b", "T4k")
FIRST_T = ("T1k", "T2k", "T3b", "T4b")     # shape [chi_E, D, chi_I]
SECOND_T = ("T1b", "T2b", "T3k", "T4k")    # shape [chi_I, D, chi_E]


def env_shapes(D: int, chi_E: int, chi_I: int) -> dict:
    """Shape of every environment tensor of one site."""
    shp = {c: (chi_E, chi_E) for c in ("C1", "C2", "C3", "C4")}
    for t in FIRST_T:
        shp[t] = (chi_E, D, chi_I)
    for t in SECOND_T:
        shp[t] = (chi_I, D, chi_E)
    return shp


def env_site_elems(D: int, chi_E: int, chi_I: int) -> int:
    return sum(int(np.prod(s)) for s in env_shapes(D, chi_E, chi_I).values())


# --------------------------------------------------------------------------
# PEPS tensors
# --------------------------------------------------------------------------
def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def peps_gaussian(seed: int, Lx: int, Ly: int, p: int, D: int) -> np.ndarray:
    """Cell of iid N(0,1) tensors, each scaled so that max|A| = 1.

    Returns an array [Lx, Ly, p, D, D, D, D] (FP64, C order)."""
    g = _rng(seed)
    A = g.standard_normal((Lx, Ly, p, D, D, D, D))
    for x in range(Lx):
        for y in range(Ly):
            A[x, y] /= np.abs(A[x, y]).max()
    return A


def peps_neel_biased(seed: int, p: int, D: int, bias: float = 0.1) -> np.ndarray:
    """1-site tensor: iid N(0,1) plus bias x a seeded Neel-like product tensor.

    The bias tensor is phi (x) e0 (x) e0 (x) e0 (x) e0 with phi a seeded spinor
    close to spin up; in the sublattice-rotated frame used for 1-site cells a
    uniform polarisation is the Neel state.  The bias is scaled to the
    Frobenius norm of the random part, so `bias` is a relative weight.  The
    result is scaled to max|A| = 1.  Shape [1, 1, p, D, D, D, D]."""
    g = _rng(seed)
    R = g.standard_normal((p, D, D, D, D))
    phi = np.zeros(p)
    phi[0] = 1.0
    phi[1:] = 0.1 * g.standard_normal(p - 1)
    phi /= np.linalg.norm(phi)
    B = np.zeros((p, D, D, D, D))
    B[:, 0, 0, 0, 0] = phi
    A = R + bias * np.linalg.norm(R) * B
    A /= np.abs(A).max()
    return A[None, None]


def peps_product(seed: int, p: int, D: int) -> np.ndarray:
    """Product state in disguise: A = phi (x) v (x) w (x) v' (x) w' (rank-1 virtual
    structure), phi a real unit spinor.  D = 1 gives a plain product state.
    Shape [1, 1, p, D, D, D, D]."""
    g = _rng(seed)
    phi = g.standard_normal(p)
    phi /= np.linalg.norm(phi)
    vs = [g.standard_normal(D) for _ in range(4)]
    A = np.einsum("p,u,l,d,r->puldr", phi, *vs)
    A /= np.abs(A).max()
    return A[None, None]


def ising_weight_sqrt(beta: float) -> np.ndarray:
    """W with (W W^T)[s,s'] = exp(beta s s' / 2), s = +1 (index 0), -1 (index 1).

    W is the symmetric square root of Q = [[e^{b/2}, e^{-b/2}], [e^{-b/2}, e^{b/2}]]."""
    Q = np.array([[np.exp(beta / 2), np.exp(-beta / 2)],
                  [np.exp(-beta / 2), np.exp(beta / 2)]])
    w, V = np.linalg.eigh(Q)
    return (V * np.sqrt(w)) @ V.T


def peps_ising(beta: float) -> np.ndarray:
    """Square-root-Boltzmann PEPS of the 2D classical Ising model (D = p = 2):
    A[s,u,l,d,r] = W[s,u] W[s,l] W[s,d] W[s,r], so <psi|psi> = Z_Ising(beta).
    Shape [1, 1, 2, 2, 2, 2, 2]."""
    W = ising_weight_sqrt(beta)
    A = np.einsum("su,sl,sd,sr->suldr", W, W, W, W)
    return A[None, None]


# --------------------------------------------------------------------------
# Hamiltonians (basis index 2 s1 + s2, spin up = 0)
# --------------------------------------------------------------------------
def heisenberg_h() -> np.ndarray:
    """S_i . S_j for spin 1/2, as a 4x4 matrix, rows (s1 s2) bra, cols ket."""
    return 0.25 * np.array([[1, 0, 0, 0],
                            [0, -1, 2, 0],
                            [0, 2, -1, 0],
                            [0, 0, 0, 1]], dtype=np.float64)


def heisenberg_h_rotated() -> np.ndarray:
    """S_i . S_j with the second spin rotated by pi about y (sublattice
    rotation); same spectrum, lets a 1-site ansatz hold Neel order."""
    return 0.25 * np.array([[-1, 0, 0, -2],
                            [0, 1, 0, 0],
                            [0, 0, 1, 0],
                            [-2, 0, 0, -1]], dtype=np.float64)


def honeycomb_heisenberg_cg() -> tuple:
    """Spin-1/2 Heisenberg model of the honeycomb lattice with two sites per
    square-lattice tensor (p = 4, physical index 2 s_a + s_b), as bond
    Hamiltonians (h_h, h_v) in the layout of heisenberg_h (rows (s1 s2) bra,
    s1 = left / upper site).  Lattice: a(c)-b(c) inside a tensor,
    b(c)-a(c + right) on horizontal bonds, a(c)-b(c + down) on vertical
    bonds; every site then has three neighbours and the smallest loops are
    hexagons.  The term inside a tensor is shared out as a quarter on each
    of its four bonds, so the energy per site of the square lattice is the
    energy per two honeycomb sites."""
    sp = np.array([[0.0, 1.0], [0.0, 0.0]])   # S^+
    sz = np.diag([0.5, -0.5])
    i2 = np.eye(2)

    def dot(x1, x2):
        # S.S = S^z S^z + (S^+ S^- + S^- S^+) / 2 between the spin that x1
        # places in the first 4-dimensional site and the one x2 places in the second
        return np.kron(x1(sz), x2(sz)) + 0.5 * (np.kron(x1(sp), x2(sp.T)) + np.kron(x1(sp.T), x2(sp)))

    on_a = lambda o: np.kron(o, i2)
    on_b = lambda o: np.kron(i2, o)
    # inside one tensor: S_a . S_b on the 4-dimensional site
    h_in = np.kron(sz, sz) + 0.5 * (np.kron(sp, sp.T) + np.kron(sp.T, sp))
    i4 = np.eye(4)
    share = 0.25 * (np.kron(h_in, i4) + np.kron(i4, h_in))
    h_h = dot(on_b, on_a) + share    # b(left) . a(right)
    h_v = dot(on_a, on_b) + share    # a(upper) . b(lower)
    return h_h, h_v


def sz_sz() -> np.ndarray:
    """sigma^z (x) sigma^z, used for the Ising nearest-neighbour correlator."""
    return np.diag([1.0, -1.0, -1.0, 1.0])


# --------------------------------------------------------------------------
# Environments
# --------------------------------------------------------------------------
def random_env(seed: int, Lx: int, Ly: int, D: int, chi_E: int, chi_I: int) -> dict:
    """Random full-rank environment: every tensor iid N(0,1) + 1 (so that the
    network has a dominant positive part and a nonzero norm), scaled to unit
    Frobenius norm.  Returns {(x, y): {name: array}}."""
    g = _rng(seed)
    shp = env_shapes(D, chi_E, chi_I)
    env = {}
    for x in range(Lx):
        for y in range(Ly):
            site = {}
            for name in ENV_NAMES:
                t = g.standard_normal(shp[name]) + 1.0
                site[name] = t / np.linalg.norm(t)
            env[(x, y)] = site
    return env


def pack_env(env: dict, Lx: int, Ly: int, D: int, chi_E: int, chi_I: int) -> np.ndarray:
    """Flat FP64 vector: sites in row-major [x][y] order, inside a site the
    twelve tensors in ENV_NAMES order, each C-contiguous at its full padded
    shape (smaller tensors are zero padded in the leading corner)."""
    shp = env_shapes(D, chi_E, chi_I)
    out = []
    for x in range(Lx):
        for y in range(Ly):
            for name in ENV_NAMES:
                t = np.asarray(env[(x, y)][name], dtype=np.float64)
                full = np.zeros(shp[name])
                full[tuple(slice(0, n) for n in t.shape)] = t
                out.append(full.ravel())
    return np.concatenate(out)


def unpack_env(flat: np.ndarray, Lx: int, Ly: int, D: int, chi_E: int, chi_I: int) -> dict:
    shp = env_shapes(D, chi_E, chi_I)
    env = {}
    off = 0
    flat = np.asarray(flat, dtype=np.float64)
    for x in range(Lx):
        for y in range(Ly):
            site = {}
            for name in ENV_NAMES:
                n = int(np.prod(shp[name]))
                site[name] = flat[off:off + n].reshape(shp[name]).copy()
                off += n
            env[(x, y)] = site
    return env


# --------------------------------------------------------------------------
# The five workloads (sizes from the benchmark definitions)
# --------------------------------------------------------------------------
WORKLOADS = {
    "d2_D2_chi8": dict(Lx=1, Ly=1, p=2, D=2, chi=8, sweeps=30, prec="fp64",
                       A="gaussian", h="rotated"),
    "d2_D4_chi32": dict(Lx=1, Ly=1, p=2, D=4, chi=32, sweeps=50, tol=1e-10,
                        prec="fp64", A="neel", h="rotated"),
    "d2_D6_chi72_grad": dict(Lx=1, Ly=1, p=2, D=6, chi=72, sweeps=40, ckpt=5,
                             prec="fp32", A="gaussian", h="rotated"),
    "cell2x2_d2_D8_chi128_grad": dict(Lx=2, Ly=2, p=2, D=8, chi=128, sweeps=None,
                                      prec="bf16x3", A="gaussian", h="plain"),
    "d2_D10_chi160_grad": dict(Lx=1, Ly=1, p=2, D=10, chi=160, sweeps=60, ckpt=5,
                               prec="bf16x3", A="gaussian", h="rotated"),
}


def workload_peps(name: str, seed: int = 1234) -> np.ndarray:
    w = WORKLOADS[name]
    if w["A"] == "neel":
        return peps_neel_biased(seed, w["p"], w["D"])
    return peps_gaussian(seed, w["Lx"], w["Ly"], w["p"], w["D"])


def workload_h(name: str) -> np.ndarray:
    return heisenberg_h_rotated() if WORKLOADS[name]["h"] == "rotated" else heisenberg_h()
