"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Every case prints what it runs before touching the GPU.  Sizes span several
MFMA tiles and ragged tails; the headline workload is covered by sampled
properties in test_gpu_workloads.py.
"""
import math

import numpy as np
import pytest
import torch

from oracle import grad as og
from oracle import split_ctmrg as sc
from paper_2502_10298_amd import binding as b
from paper_2502_10298_amd import inputs as inp

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(*a):
    print("[case]", *a, flush=True)


# ---------------------------------------------------------------------------
# kernels
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 2e-6), ("bf16x3", 4e-5), ("bf16x6", 2e-6)])
@pytest.mark.parametrize("shape", [(70, 45, 33), (300, 260, 190), (1, 129, 64), (257, 3, 1000), (200, 150, 128),
                                   (130, 70, 97), (2100, 1100, 100)])
@pytest.mark.parametrize("tA,tB", [(False, False), (True, False), (False, True), (True, True)])
def test_gemm(prec, tol, shape, tA, tB):
    M, N, K = shape
    _say("gemm", prec, shape, tA, tB)
    g = torch.Generator(device="cpu").manual_seed(M * 7 + N)
    A = torch.randn((K, M) if tA else (M, K), generator=g, dtype=torch.float64)
    B = torch.randn((N, K) if tB else (K, N), generator=g, dtype=torch.float64)
    ref = (A.T if tA else A) @ (B.T if tB else B)
    dt = torch.float64 if prec == "fp64" else torch.float32
    C = b.debug_gemm(A.to(DEV, dt), B.to(DEV, dt), tA, tB, prec).double().cpu()
    err = (C - ref).norm() / ref.norm()
    assert err < tol, float(err)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 2e-6), ("bf16x3", 4e-5), ("bf16x6", 2e-6)])
@pytest.mark.parametrize("shape", [(64, 96, 20000), (130, 7, 8193), (1, 1, 65536), (200, 100, 1500)])
@pytest.mark.parametrize("tA,tB", [(False, False), (True, False), (False, True), (True, True)])
def test_gemm_split_k(prec, tol, shape, tA, tB):
    """Long-K products with few output tiles run split over K (a ragged last
    slice included) and must equal the plain product."""
    M, N, K = shape
    assert b.lib().ctm_debug_gemm_work_bytes(b.PREC[prec], M, N, K) > 0
    _say("gemm split-k", prec, shape, tA, tB)
    g = torch.Generator(device="cpu").manual_seed(M * 11 + N)
    A = torch.randn((K, M) if tA else (M, K), generator=g, dtype=torch.float64)
    B = torch.randn((N, K) if tB else (K, N), generator=g, dtype=torch.float64)
    ref = (A.T if tA else A) @ (B.T if tB else B)
    dt = torch.float64 if prec == "fp64" else torch.float32
    C = b.debug_gemm(A.to(DEV, dt), B.to(DEV, dt), tA, tB, prec).double().cpu()
    err = (C - ref).norm() / ref.norm()
    assert err < tol, float(err)


@pytest.mark.parametrize("shape", [(1030, 1100, 1900), (2100, 2200, 700), (1024, 1024, 2048), (1500, 4100, 2000)])
@pytest.mark.parametrize("tA,tB", [(False, False), (True, False), (False, True), (True, True)])
def test_gemm_bf16x3_presplit(shape, tA, tB):
    """Large BF16X3 products run on operands split once into k-contiguous
    bf16 planes (128 x 128 tiles; ragged M, N and K; K sliced when the tiles
    are few): same bound as the in-LDS split against the FP64 product."""
    M, N, K = shape
    assert b.lib().ctm_debug_gemm_work_bytes(b.PREC["bf16x3"], M, N, K) > 0
    _say("gemm bf16x3 presplit", shape, tA, tB)
    g = torch.Generator(device="cpu").manual_seed(M * 3 + N)
    A = torch.randn((K, M) if tA else (M, K), generator=g, dtype=torch.float64)
    B = torch.randn((N, K) if tB else (K, N), generator=g, dtype=torch.float64)
    ref = (A.T if tA else A) @ (B.T if tB else B)
    C = b.debug_gemm(A.to(DEV, torch.float32), B.to(DEV, torch.float32), tA, tB, "bf16x3").double().cpu()
    err = (C - ref).norm() / ref.norm()
    assert err < 4e-5, float(err)


@pytest.mark.parametrize("n,batch", [(5, 1), (33, 2), (100, 3), (257, 1), (1024, 2)])
def test_jacobi_svd(n, batch):
    _say("svd", n, batch)
    g = torch.Generator().manual_seed(n)
    M = torch.randn(batch, n, n, generator=g, dtype=torch.float64)
    M[0, :, n // 3] = 0.0             # a zero column: rank deficient
    if n > 4:
        M[-1] = M[-1] * torch.logspace(0, -9, n, dtype=torch.float64)[None, :]   # wide spectrum
    U, S, V, sweeps = b.debug_svd(M.to(DEV))
    U, S, V = U.cpu(), S.cpu(), V.cpu()
    for i in range(batch):
        ref = torch.linalg.svdvals(M[i])
        # both decompositions are backward stable: |s - s_ref| <= c n eps s_1
        err = float((S[i] - ref).abs().max())
        assert err <= 4 * n * 2.2e-16 * float(ref[0]), err
        rec = (U[i] * S[i]) @ V[i].T
        assert (rec - M[i]).norm() < 2e-12 * math.sqrt(n / 64 + 1) * M[i].norm()
        # U S = M V and V S = M^T U have Gram matrices diag(S^2) to eps * s_1^2
        # (columns past the rank may be zero), and the singular vectors of
        # every singular value above 1e-4 s_1 are orthonormal.
        US, VS = U[i] * S[i], V[i] * S[i]
        D2 = torch.diag(S[i] ** 2)
        assert torch.allclose(US.T @ US, D2, rtol=0, atol=1e-12 * float(S[i][0]) ** 2)
        assert torch.allclose(VS.T @ VS, D2, rtol=0, atol=1e-12 * float(S[i][0]) ** 2)
        r = int((S[i] > 1e-4 * S[i][0]).sum())
        Ur, Vr = U[i][:, :r], V[i][:, :r]
        assert torch.allclose(Ur.T @ Ur, torch.eye(r, dtype=torch.float64), atol=1e-12)
        assert torch.allclose(Vr.T @ Vr, torch.eye(r, dtype=torch.float64), atol=1e-12)
        # V (the second QR's Q times the product of all Jacobi rotations) is a
        # full orthogonal matrix to working accuracy, as a Householder-based
        # SVD's is: the reverse pass of strongly graded spectra needs it (a
        # drift of 1e-13 cost 1e-6 of the gradient at chi = 48)
        assert float((V[i].T @ V[i] - torch.eye(n, dtype=torch.float64)).abs().max()) <= 5e-15 * math.sqrt(n)
    assert sweeps < 60


@pytest.mark.parametrize("n,batch", [(7, 1), (64, 2), (130, 3), (1024, 3)])
def test_jacobi_svd_full_rank(n, batch):
    """Full-rank inputs, plain and graded: the factor V of the preconditioned
    triangle R1^T is solved for by substitution after the sweeps, unless the
    check of its orthogonality sends the batch back to accumulated rotations
    (as the rank-deficient batches of test_jacobi_svd are).  The same
    accuracy either way: singular values to c n eps s_1, the reconstruction,
    both factors orthogonal to working accuracy, and the leading singular
    vectors equal to LAPACK's within eps s_1 / gap."""
    _say("svd full rank", n, batch)
    g = torch.Generator().manual_seed(1000 + n)
    M = torch.randn(batch, n, n, generator=g, dtype=torch.float64)
    if batch > 1:
        M[1] = M[1] * torch.logspace(0, -8, n, dtype=torch.float64)[None, :]   # graded columns
    if batch > 2:
        M[2] = torch.logspace(0, -6, n, dtype=torch.float64)[:, None] * M[2]   # graded rows
    U, S, V, sweeps = b.debug_svd(M.to(DEV))
    U, S, V = U.cpu(), S.cpu(), V.cpu()
    I = torch.eye(n, dtype=torch.float64)
    for i in range(batch):
        Ur, Sr, Vhr = torch.linalg.svd(M[i])
        s1 = float(Sr[0])
        assert float((S[i] - Sr).abs().max()) <= 4 * n * 2.2e-16 * s1
        rec = (U[i] * S[i]) @ V[i].T
        assert (rec - M[i]).norm() < 2e-12 * math.sqrt(n / 64 + 1) * M[i].norm()
        assert float((V[i].T @ V[i] - I).abs().max()) <= 5e-15 * math.sqrt(n)
        assert float((U[i].T @ U[i] - I).abs().max()) <= 1e-13 * math.sqrt(n)
        for j in range(min(n, 6)):
            gap = min(float(Sr[j - 1] - Sr[j]) if j > 0 else math.inf,
                      float(Sr[j] - Sr[j + 1]) if j + 1 < n else math.inf)
            bound = 100 * 2.2e-16 * s1 / gap + 1e-14
            sg = 1.0 if float(V[i][:, j] @ Vhr[j]) >= 0 else -1.0
            assert float((V[i][:, j] - sg * Vhr[j]).abs().max()) <= bound, (i, j, bound)
            assert float((U[i][:, j] - sg * Ur[:, j]).abs().max()) <= bound, (i, j, bound)
    assert sweeps < 60


@pytest.mark.parametrize("m,k,batch", [(40, 17, 1), (300, 150, 3), (2048, 1024, 2), (3200, 160, 1), (64, 64, 2),
                                       (200, 130, 2), (4096, 300, 1), (1024, 1024, 3), (2100, 200, 1),
                                       (5440, 340, 1), (8192, 100, 2)])
def test_householder_qr(m, k, batch):
    """X = Q R with Q orthonormal and R upper triangular, to working accuracy,
    on graded and rank-deficient inputs (panels of 16, 8 and 4 columns; outer
    blocks of 64 columns with a ragged last block)."""
    _say("qr", m, k, batch)
    g = torch.Generator().manual_seed(m + k)
    X = torch.randn(batch, m, k, generator=g, dtype=torch.float64)
    X[0] = X[0] * torch.logspace(0, -10, k, dtype=torch.float64)[None, :]      # graded columns
    if batch > 1:
        X[1, :, k // 2:] = X[1, :, : k - k // 2] @ torch.randn(k - k // 2, k - k // 2, generator=g,
                                                             dtype=torch.float64)   # rank k - k // 2
    Q, R = b.debug_qr(X.to(DEV))
    Q, R = Q.cpu(), R.cpu()
    for i in range(batch):
        assert torch.allclose(Q[i].T @ Q[i], torch.eye(k, dtype=torch.float64), atol=1e-13 * math.sqrt(m))
        assert (Q[i] @ R[i] - X[i]).norm() <= 1e-14 * math.sqrt(m * k) * X[i].norm()
        assert torch.equal(torch.triu(R[i]), R[i])
        # |R| diagonal equals the oracle-independent Householder result up to signs
        ref = torch.linalg.qr(X[i])[1]
        if i != 1:
            assert torch.allclose(R[i].diagonal().abs(), ref.diagonal().abs(), rtol=1e-8,
                                  atol=1e-13 * float(X[i].norm()))


# ---------------------------------------------------------------------------
# whole path, FP64, against the oracle
# ---------------------------------------------------------------------------
def _oracle_run(A_np, chi, sweeps, env0=None, alt_yr=False):
    Lx, Ly = A_np.shape[:2]
    A = sc.peps_from_numpy(A_np)
    env = sc.env_from_numpy(env0) if env0 is not None else sc.init_identity(Lx, Ly, A_np.shape[3])
    for _ in range(sweeps):
        env = sc.sweep(env, A, Lx, Ly, chi, chi, alt_yr=alt_yr)
    return env, A


def test_energy_parity_d2_chi8_fp64():
    """D=2, chi=8, 30 sweeps from the identity boundary, Heisenberg energy in
    the rotated frame: GPU FP64 equals the oracle to 1e-10 relative."""
    A_np = inp.workload_peps("d2_D2_chi8")
    h = inp.heisenberg_h_rotated()
    _say("energy d2_D2_chi8 fp64")
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), 8, prec="fp64")
    obj.sweep(30)
    e_gpu, bonds = obj.energy(h)
    env, A = _oracle_run(A_np, 8, 30)
    e_ref, bref = sc.energy(env, A, 1, 1, h)
    assert abs(e_gpu - float(e_ref)) <= 1e-10 * abs(float(e_ref)), (e_gpu, float(e_ref))
    assert abs(bonds[0, 0, 0] - float(bref[(0, 0)][0])) <= 1e-10
    assert abs(bonds[0, 0, 1] - float(bref[(0, 0)][1])) <= 1e-10


def test_env_and_projectors_parity_fp64():
    """After a few sweeps the exported environment (corner spectra) and the
    four projector pairs of every direction agree with the oracle computed
    from that same environment."""
    A_np = inp.peps_gaussian(77, 1, 1, 2, 2)
    chi = 6
    _say("projectors d2 chi6")
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), chi, prec="fp64")
    obj.sweep(3)
    flat = obj.env_export().cpu().numpy()
    env = sc.env_from_numpy(inp.unpack_env(flat, 1, 1, 2, chi, chi))
    env_ref, A = _oracle_run(A_np, chi, 3)
    for c in ("C1", "C2", "C3", "C4"):
        s_gpu = torch.linalg.svdvals(env[(0, 0)][c])
        s_ref = torch.linalg.svdvals(env_ref[(0, 0)][c])
        n = min(len(s_gpu), len(s_ref))
        assert torch.allclose(s_gpu[:n], s_ref[:n], atol=1e-11)
    for direction in range(4):
        P, te = obj.projectors(direction, 0, 0)
        e2, a2, lx, ly = sc.to_frame(["left", "top", "right", "bottom"][direction], env, A, 1, 1)
        G, Y, TH, R, _ = sc.column_projectors(e2, a2, lx, ly, 0, chi, chi)
        for nm, pr in (("green", G[0]), ("teal", TH[0]), ("yellow", Y[0]), ("red", R[0])):
            k = pr[3]
            for j, side in ((0, "_T"), (1, "_B")):
                ref = pr[j]
                got = P[nm + side].cpu()
                got = got[..., :k].reshape(ref.shape)
                scale = float(ref.abs().max())
                assert torch.allclose(got, ref, atol=1e-8 * scale, rtol=0), (direction, nm, side)
            assert float(P[nm + "_T"].cpu()[..., k:].abs().max() if k < P[nm + "_T"].shape[-1] else 0.0) == 0.0


def test_cell_2x2_parity_fp64():
    """2x2 cell of four different tensors (D=2, chi=6): every bond energy."""
    A_np = inp.peps_gaussian(91, 2, 2, 2, 2)
    h = inp.heisenberg_h()
    _say("cell2x2 d2 chi6 fp64")
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), 6, prec="fp64")
    obj.sweep(4)
    e_gpu, bonds = obj.energy(h)
    env, A = _oracle_run(A_np, 6, 4)
    e_ref, bref = sc.energy(env, A, 2, 2, h)
    assert abs(e_gpu - float(e_ref)) <= 1e-10 * abs(float(e_ref))
    for (x, y), (eh, ev) in bref.items():
        assert abs(bonds[x, y, 0] - float(eh)) <= 1e-9 and abs(bonds[x, y, 1] - float(ev)) <= 1e-9


def test_gradient_parity_fp64():
    """dE/dA from the hand-written adjoints equals the oracle's autograd
    gradient (2 sweeps from a random full-rank start, D=2, chi=4)."""
    A_np = inp.peps_gaussian(11, 1, 1, 2, 2)
    chi, ns = 4, 2
    env0 = inp.random_env(5, 1, 1, 2, chi, chi)
    h = inp.heisenberg_h_rotated()
    _say("gradient d2 chi4 fp64")
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), chi, prec="fp64", with_grad=True, n_sweeps=ns, ckpt_every=1)
    obj.env_import(torch.tensor(inp.pack_env(env0, 1, 1, 2, chi, chi), device=DEV))
    e_gpu, dA = obj.energy_grad(h, ns, 1)
    e_ref, g_ref = og.energy_and_grad(A_np, env0, chi, chi, ns, h)
    assert abs(e_gpu - e_ref) <= 1e-10 * abs(e_ref)
    g = dA.cpu().numpy()
    assert np.linalg.norm(g - g_ref) <= 1e-8 * np.linalg.norm(g_ref)


def test_gradient_checkpoint_blocks_agree():
    """Checkpointing every sweep or once for all sweeps gives the same gradient."""
    A_np = inp.peps_gaussian(12, 1, 1, 2, 2)
    chi, ns = 4, 3
    env0 = torch.tensor(inp.pack_env(inp.random_env(6, 1, 1, 2, chi, chi), 1, 1, 2, chi, chi), device=DEV)
    h = inp.heisenberg_h_rotated()
    _say("gradient checkpoint blocks")
    out = []
    for k in (1, 3, 2):
        obj = b.SplitCTM(torch.tensor(A_np, device=DEV), chi, prec="fp64", with_grad=True, n_sweeps=ns, ckpt_every=k)
        obj.env_import(env0)
        out.append(obj.energy_grad(h, ns, k))
    for e, g in out[1:]:
        assert abs(e - out[0][0]) < 1e-13
        assert torch.allclose(g, out[0][1], atol=1e-11 * float(out[0][1].abs().max()))


@pytest.mark.parametrize("ns,k", [(3, 2), (7, 5), (4, 4)])
def test_energy_grad_leaves_environment_after_n_sweeps(ns, k):
    """After ctm_energy_grad(n, k) the context holds the environment after the
    n sweeps, also when n is not a multiple of k (the last checkpoint block
    is then shorter): it equals the environment of n plain sweeps from the
    same start, and a following energy equals the energy of that state."""
    A_np = inp.peps_gaussian(12, 1, 1, 2, 2)
    chi = 4
    env0 = torch.tensor(inp.pack_env(inp.random_env(6, 1, 1, 2, chi, chi), 1, 1, 2, chi, chi), device=DEV)
    h = inp.heisenberg_h_rotated()
    _say(f"state after energy_grad({ns}, {k})")
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), chi, prec="fp64", with_grad=True, n_sweeps=ns, ckpt_every=k)
    obj.env_import(env0)
    e_grad, _ = obj.energy_grad(h, ns, k)
    after_grad = obj.env_export()
    e_after, _ = obj.energy(h)
    obj.env_import(env0)
    obj.sweep(ns)
    after_sweeps = obj.env_export()
    obj.close()
    scale = float(after_sweeps.abs().max())
    assert torch.allclose(after_grad, after_sweeps, atol=1e-13 * scale, rtol=0)
    assert abs(e_after - e_grad) <= 1e-13


def test_ctm_energy_autograd_function():
    """torch.autograd through CtmEnergy: dE/dA equals the library's
    energy_grad and the oracle's autograd gradient (D = 2, chi = 4, 2 sweeps
    from a random start, to 1e-8), and follows the upstream cotangent (the
    gradient of 3 E is 3 dE/dA)."""
    A_np = inp.peps_gaussian(11, 1, 1, 2, 2)
    chi, ns = 4, 2
    env0_np = inp.random_env(5, 1, 1, 2, chi, chi)
    env0 = torch.tensor(inp.pack_env(env0_np, 1, 1, 2, chi, chi), device=DEV)
    h = inp.heisenberg_h_rotated()
    _say("CtmEnergy autograd d2 chi4 fp64")
    A = torch.tensor(A_np, device=DEV, requires_grad=True)
    e = b.ctm_energy(A, h, chi, ns, ckpt_every=1, state={"env": env0})
    (g,) = torch.autograd.grad(e, A)
    A2 = torch.tensor(A_np, device=DEV, requires_grad=True)
    (g3,) = torch.autograd.grad(3.0 * b.ctm_energy(A2, h, chi, ns, ckpt_every=1, state={"env": env0}), A2)
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), chi, prec="fp64", with_grad=True, n_sweeps=ns, ckpt_every=1)
    obj.env_import(env0)
    e_lib, g_lib = obj.energy_grad(h, ns, 1)
    obj.close()
    e_ref, g_ref = og.energy_and_grad(A_np, env0_np, chi, chi, ns, h)
    gn = g.detach().cpu().numpy()
    assert float(e) == e_lib
    assert torch.equal(g, g_lib)
    assert abs(float(e) - e_ref) <= 1e-10 * abs(e_ref)
    assert np.linalg.norm(gn - g_ref) <= 1e-8 * np.linalg.norm(g_ref)
    assert torch.allclose(g3, 3.0 * g, rtol=1e-14, atol=0)


def test_ctm_energy_autograd_options_and_warm_start():
    """CtmEnergy passes chi_I < chi_E, a separate vertical Hamiltonian and the
    App. B alternative yellow / red flag through to the library (same result
    as SplitCTM.energy_grad with those options), and a state dict carries the
    environment from one call to the next (the second call starts where the
    first ended)."""
    A_np = inp.peps_gaussian(13, 1, 1, 2, 2)
    chiE, chiI, ns = 6, 4, 2
    h = inp.heisenberg_h_rotated()
    hv = 0.5 * inp.heisenberg_h_rotated()
    _say("CtmEnergy options d2 chiE6 chiI4 alt_yr")
    A = torch.tensor(A_np, device=DEV, requires_grad=True)
    state = {}
    e1 = b.ctm_energy(A, h, chiE, ns, chi_I=chiI, h_v=hv, alt_yr=True, state=state)
    (g1,) = torch.autograd.grad(e1, A)
    env_after_1 = state["env"].clone()
    e2 = b.ctm_energy(A, h, chiE, ns, chi_I=chiI, h_v=hv, alt_yr=True, state=state)
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), chiE, chiI, prec="fp64", with_grad=True, n_sweeps=ns,
                     ckpt_every=1, alt_yr=True)
    e_lib, g_lib = obj.energy_grad(h, ns, 1, h_v=hv)
    obj.env_import(env_after_1)
    e_lib2, _ = obj.energy_grad(h, ns, 1, h_v=hv)
    obj.close()
    assert float(e1) == e_lib and torch.equal(g1, g_lib)
    assert float(e2) == e_lib2


@pytest.mark.parametrize("L,D,chi", [(1, 4, 32), (2, 4, 32), (1, 6, 48)])
def test_gradient_parity_fp64_graded_spectra(L, D, chi):
    """dE/dA through one sweep from the environment of three sweeps (FP64),
    at sizes whose teal spectra are strongly graded (s_k / s_1 = 1e-6 at
    D = 4, chi = 32 and 2e-7 at D = 6, chi = 48): equal to the oracle's
    autograd gradient to 1e-7 relative.  The reverse pass of such a
    truncated SVD amplifies the orthogonality defect of the singular vectors
    by s_1 / s_k; with LAPACK's factors the oracle itself sits at ~1e-8
    from the exact derivative here."""
    A_np = inp.peps_gaussian(301, L, L, 2, D)
    h = inp.heisenberg_h()
    _say(f"gradient {L}x{L} D{D} chi{chi} fp64, 1 sweep from 3")
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), chi, prec="fp64", with_grad=True, n_sweeps=1, ckpt_every=1)
    obj.sweep(3)
    flat = obj.env_export()
    obj.env_import(flat)
    e_gpu, dA = obj.energy_grad(h, 1, 1)
    obj.close()
    env0 = inp.unpack_env(flat.cpu().numpy(), L, L, D, chi, chi)
    e_ref, g_ref = og.energy_and_grad(A_np, env0, chi, chi, 1, h)
    g = dA.cpu().numpy()
    err = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    print(f"[result] {L}x{L} D{D} chi{chi}: energy {abs(e_gpu - e_ref) / abs(e_ref):.1e}, gradient {err:.1e}")
    assert abs(e_gpu - e_ref) <= 1e-10 * abs(e_ref)
    assert err <= 1e-7


def test_lbfgs_steps_lower_the_energy():
    """Five L-BFGS iterations over CtmEnergy (each evaluation: 4 sweeps from
    the previous evaluation's environment, the energy and its gradient) on a
    seeded 2x2 cell of D = 2 tensors, chi = 8, FP64: the energy after the
    iterations is below the start energy, and every reported gradient is
    finite."""
    from paper_2502_10298_amd import optimize

    A0 = torch.tensor(inp.peps_gaussian(21, 2, 2, 2, 2), device=DEV)
    _say("lbfgs 2x2 D2 chi8 fp64, 5 iterations")
    A, hist = optimize.lbfgs(A0, inp.heisenberg_h(), 8, 5, n_sweeps=4, ckpt_every=4, prec="fp64", pre_sweeps=10)
    es = [r["energy"] for r in hist]
    print(f"[result] lbfgs energies: {' '.join(f'{e:.6f}' for e in es)}")
    assert all(np.isfinite(r["grad_norm"]) for r in hist)
    assert min(es) < es[0] - 1e-3
    assert es[-1] < es[0]


@pytest.fixture(scope="module")
def converged_env_d2_chi8():
    """The oracle's own environment of the d2_D2_chi8 workload after 20
    sweeps from the identity boundary (a well-conditioned start)."""
    A_np = inp.workload_peps("d2_D2_chi8")
    env, _ = _oracle_run(A_np, 8, 20)
    return A_np, {k: {n: t.detach().numpy().copy() for n, t in e.items()} for k, e in env.items()}


@pytest.mark.parametrize("prec,etol,gtol", [("fp64", 1e-10, 1e-8), ("fp32", 1e-6, 1e-5), ("bf16x6", 1e-6, 1e-5),
                                            ("bf16x3", 5e-5, 5e-4)])
def test_mixed_precision_gradient(prec, etol, gtol, converged_env_d2_chi8):
    """Energy and dE/dA (2 sweeps from a converged start, D=2, chi=8) with
    FP32 / BF16x6 contractions and FP64 projectors and decomposition
    adjoints, against the oracle's autograd gradient: energy to 1e-6 and
    gradient to 1e-5 relative.  BF16x3 is held to what its 2^-17 operand
    split allows (5e-5, 5e-4)."""
    A_np, env0 = converged_env_d2_chi8
    chi, ns = 8, 2
    h = inp.heisenberg_h_rotated()
    _say("gradient d2 chi8 from a converged start", prec)
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), chi, prec=prec, with_grad=True, n_sweeps=ns, ckpt_every=1)
    obj.env_import(torch.tensor(inp.pack_env(env0, 1, 1, 2, chi, chi), device=DEV))
    e_gpu, dA = obj.energy_grad(h, ns, 1)
    e_ref, g_ref = og.energy_and_grad(A_np, env0, chi, chi, ns, h)
    g = dA.cpu().numpy()
    eerr = abs(e_gpu - e_ref) / abs(e_ref)
    gerr = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    print(f"[result] {prec}: energy rel err {eerr:.2e}, gradient rel err {gerr:.2e}", flush=True)
    assert eerr <= etol, eerr
    assert gerr <= gtol, gerr


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-6), ("bf16x6", 1e-6), ("bf16x3", 5e-5)])
def test_mixed_precision_energy(prec, tol):
    """FP32 contractions and BF16x6 (three-way bf16 split, six products) with
    FP64 projectors: energy within 1e-6 relative of the FP64 oracle.  BF16x3
    (two-term split, three products) carries a 2^-17 operand error; its
    measured energy error is about 1.3e-5."""
    A_np = inp.workload_peps("d2_D2_chi8")
    h = inp.heisenberg_h_rotated()
    _say("energy d2_D2_chi8", prec)
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), 8, prec=prec)
    obj.sweep(30)
    e_gpu, _ = obj.energy(h)
    env, A = _oracle_run(A_np, 8, 30)
    e_ref, _ = sc.energy(env, A, 1, 1, h)
    assert abs(e_gpu - float(e_ref)) <= tol * abs(float(e_ref)), (e_gpu, float(e_ref))


def test_energy_parity_honeycomb_p4_fp64():
    """Honeycomb Heisenberg model with two sites per tensor (p = 4): separate
    horizontal and vertical bond Hamiltonians, neither symmetric under exchange
    of the two tensors.  1 x 2 cell of different Gaussian tensors, D = 2,
    chi = 6, 10 sweeps: GPU FP64 energy and every bond energy equal the oracle's."""
    A_np = inp.peps_gaussian(404, 1, 2, 4, 2)
    h_h, h_v = inp.honeycomb_heisenberg_cg()
    _say("energy honeycomb p=4 cell1x2 D2 chi6 fp64")
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), 6, prec="fp64")
    obj.sweep(10)
    e_gpu, bonds = obj.energy(h_h, h_v)
    env, A = _oracle_run(A_np, 6, 10)
    e_ref, bref = sc.energy(env, A, 1, 2, h_h, h_v)
    assert abs(e_gpu - float(e_ref)) <= 1e-10 * abs(float(e_ref)), (e_gpu, float(e_ref))
    for (x, y), (eh, ev) in bref.items():
        assert abs(bonds[x, y, 0] - float(eh)) <= 1e-9 and abs(bonds[x, y, 1] - float(ev)) <= 1e-9
    # one Hamiltonian for both directions is the plain entry point
    e1, _ = obj.energy(h_h)
    e2, _ = obj.energy(h_h, h_h)
    assert e1 == e2


def test_gradient_parity_honeycomb_p4_fp64():
    """dE/dA of the p = 4 honeycomb model (separate horizontal and vertical
    bond Hamiltonians) equals the oracle's autograd gradient: D = 2, chi = 4,
    2 sweeps from the oracle's own environment after 10 sweeps (a random
    start puts near-degenerate singular values at the cut, where the two
    sides' roundings already differ by 1e-9 in the energy)."""
    A_np = inp.peps_gaussian(405, 1, 1, 4, 2)
    chi, ns = 4, 2
    env_c, _ = _oracle_run(A_np, chi, 10)
    env0 = {k: {n: t.detach().numpy().copy() for n, t in e.items()} for k, e in env_c.items()}
    h_h, h_v = inp.honeycomb_heisenberg_cg()
    _say("gradient honeycomb p=4 D2 chi4 fp64")
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), chi, prec="fp64", with_grad=True, n_sweeps=ns, ckpt_every=1)
    obj.env_import(torch.tensor(inp.pack_env(env0, 1, 1, 2, chi, chi), device=DEV))
    e_gpu, dA = obj.energy_grad(h_h, ns, 1, h_v=h_v)
    e_ref, g_ref = og.energy_and_grad(A_np, env0, chi, chi, ns, h_h, h_v=h_v)
    assert abs(e_gpu - e_ref) <= 1e-10 * abs(e_ref)
    g = dA.cpu().numpy()
    assert np.linalg.norm(g - g_ref) <= 1e-8 * np.linalg.norm(g_ref)


# ---------------------------------------------------------------------------
# error paths (forced from the host; every kernel exits normally)
# ---------------------------------------------------------------------------
def test_workspace_too_small_is_einval():
    A = torch.tensor(inp.peps_gaussian(1, 1, 1, 2, 2), device=DEV)
    _say("workspace too small")
    with pytest.raises(b.CtmError) as ei:
        b.SplitCTM(A, 8, workspace_bytes=1024)
    assert ei.value.status == b.CTM_EINVAL


@pytest.mark.parametrize("alt_yr,half_teal", [(False, False), (True, False), (False, True), (True, True)])
@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
@pytest.mark.parametrize("D", [1, 2])
def test_product_states_exact_energy(D, prec, alt_yr, half_teal):
    """Degenerate input: a product state in disguise (rank-1 virtual
    structure, D = 1 a plain product state) with chi = 6, so every projector
    matrix has rank one and the Jacobi, the truncation and the rank-limited
    route run on spectra that are zero past the first value.  Each bond
    gives exactly +1/4 for S.S and -1/4 in the rotated frame (the oracle's
    closed-form pin, every projector construction), to rounding in FP64 and
    within the BF16x3 bounds of the other tests (5e-5 energy, 5e-4
    gradient); the environment stays finite.  The
    state is an eigenvector of H (every spin along the same axis: each bond
    at the top of the S.S spectrum), a stationary point of the energy, so
    the gradient two sweeps on vanishes to rounding (FP64) or to the split's
    error (BF16x3)."""
    _say("product state", D, prec, alt_yr, half_teal)
    A_np = inp.peps_product(3 + D, 2, D)
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), 6, 6, prec=prec, alt_yr=alt_yr, half_teal=half_teal,
                     with_grad=True, n_sweeps=2, ckpt_every=2)
    obj.sweep(4)
    e, _ = obj.energy(inp.heisenberg_h())
    e2, _ = obj.energy(inp.heisenberg_h_rotated())
    tol = 1e-12 if prec == "fp64" else 5e-5   # BF16x3: the bound of its other energy tests (2^-17 operands)
    assert abs(e - 0.5) < tol, e
    assert abs(e2 + 0.5) < tol, e2
    assert torch.isfinite(obj.env_export()).all()
    eg, g = obj.energy_grad(inp.heisenberg_h(), 2, 2)
    g = g.cpu().numpy()
    obj.close()
    assert abs(eg - 0.5) < tol and np.isfinite(g).all()
    gn = float(np.linalg.norm(g))
    print(f"[result] product state D={D} {prec} alt_yr={alt_yr} half_teal={half_teal}: E {e:.15f}, "
          f"rotated {e2:.15f}, |dE/dA| {gn:.2e} (|A| {np.linalg.norm(A_np):.2f})")
    assert gn <= (1e-12 if prec == "fp64" else 5e-4) * np.linalg.norm(A_np)


def test_nan_input_is_enumeric():
    A_np = inp.peps_gaussian(2, 1, 1, 2, 2)
    A_np[0, 0, 0, 0, 0, 0, 0] = np.nan
    _say("nan input")
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), 6)
    st, n, d = obj.sweep(2, tol=1e-8, check=False)
    assert st == b.CTM_ENUMERIC


def test_not_converged_is_reported():
    A_np = inp.peps_gaussian(3, 1, 1, 2, 2)
    _say("not converged")
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), 6)
    st, n, d = obj.sweep(1, tol=1e-300, check=False)
    assert st == b.CTM_ENOTCONV and n == 1
    e, _ = obj.energy(inp.heisenberg_h())   # environment still usable
    assert math.isfinite(e)


def test_kernel_timing_sampling():
    """Sampled event timing counts every launch and its work, and its time
    estimate (sampled mean x launches) agrees with timing every launch."""
    A = torch.tensor(inp.workload_peps("d2_D2_chi8"), device=DEV)
    _say("kernel timing sampling")
    obj = b.SplitCTM(A, 8, prec="fp64")
    obj.sweep(3)
    env = obj.env_export()
    res = {}
    for stride in (1, 4):
        obj.env_import(env)
        torch.cuda.synchronize()
        obj.kernel_timing_enable(True, stride=stride)
        obj.sweep(3)
        res[stride] = obj.kernel_timing()
        obj.kernel_timing_enable(False)
    for k in ("gemm_fp64", "jacobi_pair", "jacobi_rotate"):
        ms1, n1, f1, b1 = res[1][k]
        ms4, n4, f4, b4 = res[4][k]
        assert n1 == n4 > 0 and f1 == f4 and b1 == b4, k
        assert ms1 > 0 and 0.5 * ms1 < ms4 < 2.0 * ms1, (k, ms1, ms4)
    with pytest.raises(b.CtmError):
        obj.kernel_timing_enable(True, stride=-1)
    obj.close()


def test_energy_parity_chiI_below_chiE_fp64():
    """Independent interlayer bond chi_I < chi_E (D=2, chi_E=8, chi_I=4, 20
    sweeps): GPU FP64 energy and corner spectra equal the oracle's."""
    A_np = inp.workload_peps("d2_D2_chi8")
    h = inp.heisenberg_h_rotated()
    ce, ci, ns = 8, 4, 20
    _say("energy chi_E=8 chi_I=4 fp64")
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), ce, ci, prec="fp64")
    obj.sweep(ns)
    e_gpu, _ = obj.energy(h)
    A = sc.peps_from_numpy(A_np)
    env = sc.init_identity(1, 1, A_np.shape[3])
    for _ in range(ns):
        env = sc.sweep(env, A, 1, 1, ce, ci)
    e_ref, _ = sc.energy(env, A, 1, 1, h)
    assert abs(e_gpu - float(e_ref)) <= 1e-10 * abs(float(e_ref)), (e_gpu, float(e_ref))
    flat = obj.env_export().cpu().numpy()
    env_gpu = sc.env_from_numpy(inp.unpack_env(flat, 1, 1, 2, ce, ci))
    for c in ("C1", "C2", "C3", "C4"):
        s_gpu = torch.linalg.svdvals(env_gpu[(0, 0)][c])
        s_ref = torch.linalg.svdvals(env[(0, 0)][c])
        n = min(len(s_gpu), len(s_ref))
        assert torch.allclose(s_gpu[:n], s_ref[:n], atol=1e-11)


def test_gradient_parity_chiI_below_chiE_fp64():
    """dE/dA with chi_E = 6, chi_I = 4 (2 sweeps from the oracle's environment
    after 10 sweeps from the identity boundary) equals the oracle's autograd
    gradient."""
    A_np = inp.workload_peps("d2_D2_chi8")
    ce, ci, ns = 6, 4, 2
    A = sc.peps_from_numpy(A_np)
    env = sc.init_identity(1, 1, A_np.shape[3])
    for _ in range(10):
        env = sc.sweep(env, A, 1, 1, ce, ci)
    env0 = {k: {n: t.detach().numpy().copy() for n, t in e.items()} for k, e in env.items()}
    h = inp.heisenberg_h_rotated()
    _say("gradient chi_E=6 chi_I=4 fp64")
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), ce, ci, prec="fp64", with_grad=True, n_sweeps=ns, ckpt_every=1)
    obj.env_import(torch.tensor(inp.pack_env(env0, 1, 1, 2, ce, ci), device=DEV))
    e_gpu, dA = obj.energy_grad(h, ns, 1)
    e_ref, g_ref = og.energy_and_grad(A_np, env0, ce, ci, ns, h)
    assert abs(e_gpu - e_ref) <= 1e-10 * abs(e_ref)
    g = dA.cpu().numpy()
    assert np.linalg.norm(g - g_ref) <= 1e-8 * np.linalg.norm(g_ref)


# ---------------------------------------------------------------------------
# App. B constructions: alternative yellow / red projectors (physical leg cut
# by yellow) and teal half projectors (left halves of the patch), alone and
# combined
# ---------------------------------------------------------------------------
APP_B = [(True, False), (False, True), (True, True)]


def _oracle_run_v(A_np, chi, sweeps, alt_yr, half_teal):
    Lx, Ly = A_np.shape[:2]
    A = sc.peps_from_numpy(A_np)
    env = sc.init_identity(Lx, Ly, A_np.shape[3])
    for _ in range(sweeps):
        env = sc.sweep(env, A, Lx, Ly, chi, chi, alt_yr=alt_yr, half_teal=half_teal)
    return env, A


@pytest.mark.parametrize("alt_yr,half_teal", APP_B)
def test_app_b_energy_parity_fp64(alt_yr, half_teal):
    """D=2, chi=8, 20 sweeps from the identity boundary with the App. B
    constructions: GPU FP64 equals the oracle to 1e-10."""
    A_np = inp.workload_peps("d2_D2_chi8")
    h = inp.heisenberg_h_rotated()
    _say("app_b energy d2_D2_chi8 fp64", alt_yr, half_teal)
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), 8, prec="fp64", alt_yr=alt_yr, half_teal=half_teal)
    obj.sweep(20)
    e_gpu, bonds = obj.energy(h)
    env, A = _oracle_run_v(A_np, 8, 20, alt_yr, half_teal)
    e_ref, bref = sc.energy(env, A, 1, 1, h)
    assert abs(e_gpu - float(e_ref)) <= 1e-10 * abs(float(e_ref)), (e_gpu, float(e_ref))
    assert abs(bonds[0, 0, 0] - float(bref[(0, 0)][0])) <= 1e-10
    assert abs(bonds[0, 0, 1] - float(bref[(0, 0)][1])) <= 1e-10


@pytest.mark.parametrize("alt_yr,half_teal", APP_B)
def test_app_b_cell_2x2_parity_fp64(alt_yr, half_teal):
    """2x2 cell of four different tensors (D=2, chi=6), App. B constructions:
    every bond energy."""
    A_np = inp.peps_gaussian(91, 2, 2, 2, 2)
    h = inp.heisenberg_h()
    _say("app_b cell2x2 d2 chi6 fp64", alt_yr, half_teal)
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), 6, prec="fp64", alt_yr=alt_yr, half_teal=half_teal)
    obj.sweep(4)
    e_gpu, bonds = obj.energy(h)
    env, A = _oracle_run_v(A_np, 6, 4, alt_yr, half_teal)
    e_ref, bref = sc.energy(env, A, 2, 2, h)
    assert abs(e_gpu - float(e_ref)) <= 1e-10 * abs(float(e_ref))
    for (x, y), (eh, ev) in bref.items():
        assert abs(bonds[x, y, 0] - float(eh)) <= 1e-9 and abs(bonds[x, y, 1] - float(ev)) <= 1e-9


@pytest.mark.parametrize("alt_yr,half_teal", APP_B)
def test_app_b_projectors_parity_fp64(alt_yr, half_teal):
    """The four projector pairs of every direction (with ALT_YR: yellow
    [chi_I, D, p, chi_I], red [chi_I, D, chi_I]) agree with the oracle's from
    the same environment."""
    A_np = inp.peps_gaussian(77, 1, 1, 2, 2)
    chi = 6
    _say("app_b projectors d2 chi6", alt_yr, half_teal)
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), chi, prec="fp64", alt_yr=alt_yr, half_teal=half_teal)
    obj.sweep(3)
    flat = obj.env_export().cpu().numpy()
    env = sc.env_from_numpy(inp.unpack_env(flat, 1, 1, 2, chi, chi))
    A = sc.peps_from_numpy(A_np)
    for direction in range(4):
        P, te = obj.projectors(direction, 0, 0)
        e2, a2, lx, ly = sc.to_frame(["left", "top", "right", "bottom"][direction], env, A, 1, 1)
        G, Y, TH, R, _ = sc.column_projectors(e2, a2, lx, ly, 0, chi, chi, alt_yr=alt_yr, half_teal=half_teal)
        if alt_yr:
            assert Y[0][0].shape[:3] == (chi, 2, 2) and R[0][0].dim() == 3
        for nm, pr in (("green", G[0]), ("teal", TH[0]), ("yellow", Y[0]), ("red", R[0])):
            k = pr[3]
            for j, side in ((0, "_T"), (1, "_B")):
                ref = pr[j]
                got = P[nm + side].cpu()
                got = got[..., :k].reshape(ref.shape)
                scale = float(ref.abs().max())
                assert torch.allclose(got, ref, atol=1e-8 * scale, rtol=0), (direction, nm, side)


@pytest.mark.parametrize("alt_yr,half_teal", APP_B)
def test_app_b_gradient_parity_fp64(alt_yr, half_teal):
    """dE/dA through the App. B constructions (hand-written adjoints) equals
    the oracle's autograd gradient (2 sweeps from a random start)."""
    A_np = inp.peps_gaussian(11, 1, 1, 2, 2)
    chi, ns = 4, 2
    env0 = inp.random_env(5, 1, 1, 2, chi, chi)
    h = inp.heisenberg_h_rotated()
    _say("app_b gradient d2 chi4 fp64", alt_yr, half_teal)
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), chi, prec="fp64", with_grad=True, n_sweeps=ns, ckpt_every=1,
                     alt_yr=alt_yr, half_teal=half_teal)
    obj.env_import(torch.tensor(inp.pack_env(env0, 1, 1, 2, chi, chi), device=DEV))
    e_gpu, dA = obj.energy_grad(h, ns, 1)
    e_ref, g_ref = og.energy_and_grad(A_np, env0, chi, chi, ns, h, alt_yr=alt_yr, half_teal=half_teal)
    assert abs(e_gpu - e_ref) <= 1e-10 * abs(e_ref)
    g = dA.cpu().numpy()
    assert np.linalg.norm(g - g_ref) <= 1e-8 * np.linalg.norm(g_ref)


@pytest.mark.parametrize("prec,tol", [("fp32", 5e-6), ("bf16x6", 1e-6), ("bf16x3", 5e-5)])
@pytest.mark.parametrize("alt_yr,half_teal", APP_B)
def test_app_b_mixed_precision_energy(prec, tol, alt_yr, half_teal):
    """The App. B constructions with reduced-precision contractions (FP64
    projectors) against the FP64 oracle of the same construction.  Measured
    relative energy errors (alt / half / both): FP32 1.9e-6 / 1.8e-7 / 2.0e-7,
    BF16x6 2.4e-7 / 2.9e-7 / 1.5e-7, BF16x3 5.8e-6 / 5.2e-6 / 7.5e-6; the
    alternative yellow / red is the most sensitive to FP32 rounding, hence
    the FP32 bound of 5e-6 (1e-6 for App. A)."""
    A_np = inp.workload_peps("d2_D2_chi8")
    h = inp.heisenberg_h_rotated()
    _say("app_b energy d2_D2_chi8", prec, alt_yr, half_teal)
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), 8, prec=prec, alt_yr=alt_yr, half_teal=half_teal)
    obj.sweep(30)
    e_gpu, _ = obj.energy(h)
    env, A = _oracle_run_v(A_np, 8, 30, alt_yr, half_teal)
    e_ref, _ = sc.energy(env, A, 1, 1, h)
    assert abs(e_gpu - float(e_ref)) <= tol * abs(float(e_ref)), (e_gpu, float(e_ref))


@pytest.fixture(scope="module")
def converged_env_d2_chi8_alt():
    """The oracle's environment of the d2_D2_chi8 workload after 20 sweeps
    with the alternative yellow / red projectors of App. B."""
    A_np = inp.workload_peps("d2_D2_chi8")
    env, _ = _oracle_run_v(A_np, 8, 20, True, False)
    return A_np, {k: {n: t.detach().numpy().copy() for n, t in e.items()} for k, e in env.items()}


@pytest.mark.parametrize("prec,etol,gtol", [("fp64", 1e-10, 1e-8), ("fp32", 1e-6, 1e-5), ("bf16x6", 1e-6, 1e-5),
                                            ("bf16x3", 5e-5, 5e-4)])
def test_app_b_mixed_precision_gradient(prec, etol, gtol, converged_env_d2_chi8_alt):
    """Energy and dE/dA through the alternative yellow / red projectors (2
    sweeps from the oracle's converged start, D=2, chi=8) with reduced-
    precision contractions against the FP64 oracle of the same construction,
    to the bounds of the App. A test.  Measured (energy, gradient): FP64
    2.1e-14, 2.6e-10; FP32 1.4e-8, 1.2e-6; BF16x6 3.0e-7, 5.5e-7; BF16x3
    1.5e-5, 3.2e-5."""
    A_np, env0 = converged_env_d2_chi8_alt
    chi, ns = 8, 2
    h = inp.heisenberg_h_rotated()
    _say("app_b gradient d2 chi8 from a converged start", prec)
    obj = b.SplitCTM(torch.tensor(A_np, device=DEV), chi, prec=prec, with_grad=True, n_sweeps=ns, ckpt_every=1,
                     alt_yr=True)
    obj.env_import(torch.tensor(inp.pack_env(env0, 1, 1, 2, chi, chi), device=DEV))
    e_gpu, dA = obj.energy_grad(h, ns, 1)
    e_ref, g_ref = og.energy_and_grad(A_np, env0, chi, chi, ns, h, alt_yr=True)
    g = dA.cpu().numpy()
    eerr = abs(e_gpu - e_ref) / abs(e_ref)
    gerr = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    print(f"[result] {prec}: energy rel err {eerr:.2e}, gradient rel err {gerr:.2e}", flush=True)
    assert eerr <= etol, eerr
    assert gerr <= gtol, gerr
