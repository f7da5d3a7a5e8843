"""Thin Python binding of libsplitctm.so (C ABI of include/splitctm.h).

Argument marshalling only: every step of the split-CTMRG path runs in the
library's HIP kernels.  PyTorch provides device memory and the stream.  The
library must be built (python -m paper_2502_10298_amd.build); importing this
module without it raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsplitctm.so")

CTM_OK, CTM_EINVAL, CTM_ENOMEM, CTM_EDEVICE, CTM_ENOTCONV, CTM_ENUMERIC = range(6)
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}
INIT = {"identity": 0, "product": 1}

EXPORTED = ("ctm_workspace_size", "ctm_init", "ctm_sweep", "ctm_projectors", "ctm_projectors_elems",
            "ctm_move_column", "ctm_init_static",
            "ctm_energy", "ctm_energy_grad", "ctm_env_elems", "ctm_env_export", "ctm_env_import",
            "ctm_energy_hv", "ctm_energy_grad_hv", "ctm_last_stats", "ctm_debug_gemm_work_bytes", "ctm_debug_gemm", "ctm_debug_svd_work_bytes", "ctm_debug_svd", "ctm_debug_qr_work_bytes", "ctm_debug_qr",
            "ctm_kernel_timing_enable", "ctm_kernel_timing", "ctm_destroy", "ctm_strerror")
KERNEL_CLASSES = {"gemm_fp64": 0, "gemm_fp32": 1, "gemm_bf16x3": 2, "jacobi_pair": 3,
                  "jacobi_rotate": 5, "gemm_bf16x6": 6}


class CtmError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {strerror(status)} (status {status})")
        self.status = status


class ctm_config(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int), ("Ly", ctypes.c_int), ("p", ctypes.c_int), ("D", ctypes.c_int),
                ("chi_E", ctypes.c_int), ("chi_I", ctypes.c_int), ("contract_prec", ctypes.c_int),
                ("svd_rel_cutoff", ctypes.c_double), ("svd_adj_eps", ctypes.c_double), ("init", ctypes.c_int),
                ("projector_variant", ctypes.c_int)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libsplitctm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2502_10298_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    cfgp = ctypes.POINTER(ctm_config)
    sig = {
        "ctm_workspace_size": (I, [cfgp, I, I, I, ctypes.POINTER(S)]),
        "ctm_init": (I, [cfgp, P, P, P, S, P, ctypes.POINTER(P)]),
        "ctm_init_static": (I, [cfgp, P, P, P, ctypes.POINTER(P)]),
        "ctm_sweep": (I, [P, I, D, ctypes.POINTER(I), ctypes.POINTER(D)]),
        "ctm_projectors": (I, [P, I, I, I, P, P]),
        "ctm_projectors_elems": (S, [cfgp]),
        "ctm_move_column": (I, [P, I, I]),
        "ctm_energy": (I, [P, P, ctypes.POINTER(D), P]),
        "ctm_energy_grad": (I, [P, P, I, I, ctypes.POINTER(D), P]),
        "ctm_energy_hv": (I, [P, P, P, ctypes.POINTER(D), P]),
        "ctm_energy_grad_hv": (I, [P, P, P, I, I, ctypes.POINTER(D), P]),
        "ctm_env_elems": (S, [cfgp]),
        "ctm_env_export": (I, [P, P]),
        "ctm_env_import": (I, [P, P]),
        "ctm_last_stats": (I, [P, ctypes.POINTER(D), ctypes.POINTER(D)]),
        "ctm_debug_gemm_work_bytes": (S, [I, I, I, I]),
        "ctm_debug_gemm": (I, [I, I, I, I, I, I, P, P, P, P, P]),
        "ctm_debug_svd_work_bytes": (S, [I, I]),
        "ctm_debug_svd": (I, [I, I, P, P, P, P, P, ctypes.POINTER(I), P]),
        "ctm_debug_qr_work_bytes": (S, [I, I, I]),
        "ctm_debug_qr": (I, [I, I, I, P, P, P, P, P]),
        "ctm_kernel_timing_enable": (I, [P, I]),
        "ctm_kernel_timing": (I, [P, I, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D)]),
        "ctm_destroy": (None, [P]),
        "ctm_strerror": (ctypes.c_char_p, [I]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def strerror(status: int) -> str:
    return lib().ctm_strerror(status).decode()


def make_config(Lx, Ly, p, D, chi_E, chi_I, prec="fp64", init="identity", cutoff=1e-12, adj_eps=1e-12,
                alt_yr=False, half_teal=False):
    """alt_yr / half_teal: the alternative yellow / red projectors and the
    teal half projectors of App. B (they combine)."""
    return ctm_config(Lx, Ly, p, D, chi_E, chi_I, PREC[prec], cutoff, adj_eps, INIT[init],
                      (1 if alt_yr else 0) | (2 if half_teal else 0))


def workspace_size(cfg: ctm_config, with_grad=False, n_sweeps=0, ckpt_every=1) -> int:
    out = ctypes.c_size_t(0)
    st = lib().ctm_workspace_size(ctypes.byref(cfg), int(with_grad), n_sweeps, ckpt_every, ctypes.byref(out))
    if st != CTM_OK:
        raise CtmError(st, "ctm_workspace_size")
    return out.value


def _stream_ptr(torch, stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class SplitCTM:
    """One split-CTMRG context on the current HIP device.

    A: torch FP64 tensor [Lx, Ly, p, D, D, D, D] on the GPU (copied at init).
    alt_yr / half_teal: the alternative yellow / red projectors and the teal
    half projectors of App. B.  static_workspace: the context works in the
    library's static device array (ctm_init_static) and no workspace is
    allocated here."""

    def __init__(self, A, chi_E, chi_I=None, prec="fp64", init="identity", boundary=None,
                 with_grad=False, n_sweeps=0, ckpt_every=1, cutoff=1e-12, adj_eps=1e-12,
                 workspace_bytes=None, stream=None, alt_yr=False, half_teal=False, static_workspace=False):
        self.torch = torch
        if A.dtype != torch.float64 or not A.is_cuda or A.dim() != 7:
            raise ValueError("A must be a CUDA float64 tensor [Lx, Ly, p, D, D, D, D]")
        Lx, Ly, p, D = A.shape[:4]
        self.cfg = make_config(Lx, Ly, p, D, chi_E, chi_I if chi_I is not None else chi_E, prec, init,
                               cutoff, adj_eps, alt_yr, half_teal)
        if static_workspace:
            self.ws_bytes, self.ws = 0, None
        else:
            need = workspace_size(self.cfg, with_grad, n_sweeps, ckpt_every)
            self.ws_bytes = int(workspace_bytes) if workspace_bytes is not None else need
            self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=A.device)
        self.stream = stream
        self.A = A.contiguous()
        bvec = None
        if init == "product":
            self._bvec = (ctypes.c_double * D)(*[float(v) for v in np.asarray(boundary, dtype=np.float64)])
            bvec = ctypes.cast(self._bvec, ctypes.c_void_p)
        h = ctypes.c_void_p()
        if static_workspace:
            st = lib().ctm_init_static(ctypes.byref(self.cfg), _ptr(self.A), bvec, _stream_ptr(torch, stream),
                                       ctypes.byref(h))
        else:
            st = lib().ctm_init(ctypes.byref(self.cfg), _ptr(self.A), bvec, _ptr(self.ws),
                                ctypes.c_size_t(self.ws_bytes), _stream_ptr(torch, stream), ctypes.byref(h))
        if st != CTM_OK:
            raise CtmError(st, "ctm_init_static" if static_workspace else "ctm_init")
        self.h = h
        self.env_elems = lib().ctm_env_elems(ctypes.byref(self.cfg))

    def close(self):
        if getattr(self, "h", None):
            lib().ctm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, max_sweeps, tol=0.0, check=True):
        n = ctypes.c_int(0)
        d = ctypes.c_double(0.0)
        st = lib().ctm_sweep(self.h, max_sweeps, tol, ctypes.byref(n), ctypes.byref(d))
        if check and st not in (CTM_OK, CTM_ENOTCONV):
            raise CtmError(st, "ctm_sweep")
        return st, n.value, d.value

    def move_column(self, direction, y):
        """One column of one directional move (ctm_move_column)."""
        st = lib().ctm_move_column(self.h, direction, y)
        if st != CTM_OK:
            raise CtmError(st, "ctm_move_column")

    def energy(self, h, h_v=None):
        """Energy per site; h on horizontal bonds, h_v (default h) on vertical ones."""
        hh = np.ascontiguousarray(h, dtype=np.float64)
        hv = hh if h_v is None else np.ascontiguousarray(h_v, dtype=np.float64)
        if hv.shape != hh.shape:
            raise ValueError("h and h_v must have the same shape")
        e = ctypes.c_double(0.0)
        bonds = np.zeros((self.cfg.Lx, self.cfg.Ly, 2))
        st = lib().ctm_energy_hv(self.h, hh.ctypes.data_as(ctypes.c_void_p), hv.ctypes.data_as(ctypes.c_void_p),
                                 ctypes.byref(e), bonds.ctypes.data_as(ctypes.c_void_p))
        if st != CTM_OK:
            raise CtmError(st, "ctm_energy_hv")
        return e.value, bonds

    def projectors(self, direction, x, y):
        torch = self.torch
        n = lib().ctm_projectors_elems(ctypes.byref(self.cfg))
        out = torch.zeros(n, dtype=torch.float64, device=self.A.device)
        te = np.zeros(4)
        st = lib().ctm_projectors(self.h, direction, x, y, _ptr(out), te.ctypes.data_as(ctypes.c_void_p))
        if st != CTM_OK:
            raise CtmError(st, "ctm_projectors")
        c = self.cfg
        if c.projector_variant & 1:   # App. B: the physical leg is cut by yellow
            shapes = [(c.chi_E, c.D, c.chi_E)] * 4 + [(c.chi_I, c.D, c.p, c.chi_I)] * 2 + [(c.chi_I, c.D, c.chi_I)] * 2
        else:
            shapes = [(c.chi_E, c.D, c.chi_E)] * 4 + [(c.chi_I, c.D, c.chi_I)] * 2 + [(c.chi_I, c.p, c.D, c.chi_I)] * 2
        names = ["green_T", "green_B", "teal_T", "teal_B", "yellow_T", "yellow_B", "red_T", "red_B"]
        res, off = {}, 0
        for nm, sh in zip(names, shapes):
            k = int(np.prod(sh))
            res[nm] = out[off:off + k].reshape(sh)
            off += k
        return res, te

    def energy_grad(self, h, n_sweeps, ckpt_every=1, h_v=None):
        torch = self.torch
        hh = np.ascontiguousarray(h, dtype=np.float64)
        hv = hh if h_v is None else np.ascontiguousarray(h_v, dtype=np.float64)
        if hv.shape != hh.shape:
            raise ValueError("h and h_v must have the same shape")
        e = ctypes.c_double(0.0)
        dA = torch.zeros_like(self.A)
        st = lib().ctm_energy_grad_hv(self.h, hh.ctypes.data_as(ctypes.c_void_p), hv.ctypes.data_as(ctypes.c_void_p),
                                      n_sweeps, ckpt_every, ctypes.byref(e), _ptr(dA))
        if st != CTM_OK:
            raise CtmError(st, "ctm_energy_grad_hv")
        return e.value, dA

    def env_export(self):
        torch = self.torch
        out = torch.zeros(self.env_elems, dtype=torch.float64, device=self.A.device)
        st = lib().ctm_env_export(self.h, _ptr(out))
        if st != CTM_OK:
            raise CtmError(st, "ctm_env_export")
        return out

    def env_import(self, flat):
        flat = flat.to(dtype=self.torch.float64).contiguous()
        if flat.numel() != self.env_elems:
            raise ValueError("environment size mismatch")
        st = lib().ctm_env_import(self.h, _ptr(flat))
        if st != CTM_OK:
            raise CtmError(st, "ctm_env_import")

    def kernel_timing_enable(self, on=True, stride=1):
        """Event timing of every `stride`-th launch per kernel class (off: on=False)."""
        st = lib().ctm_kernel_timing_enable(self.h, int(stride) if on else 0)
        if st != CTM_OK:
            raise CtmError(st, "ctm_kernel_timing_enable")

    def kernel_timing(self):
        """{class: (ms, launches, flops, bytes)} summed since kernel_timing_enable."""
        out = {}
        for name, k in KERNEL_CLASSES.items():
            v = [ctypes.c_double(0) for _ in range(4)]
            st = lib().ctm_kernel_timing(self.h, k, *[ctypes.byref(x) for x in v])
            if st != CTM_OK:
                raise CtmError(st, "ctm_kernel_timing")
            out[name] = tuple(x.value for x in v)
        return out

    def stats(self):
        f = ctypes.c_double(0)
        s = ctypes.c_double(0)
        lib().ctm_last_stats(self.h, ctypes.byref(f), ctypes.byref(s))
        return f.value, s.value


def debug_gemm(A, B, transA=False, transB=False, prec="fp64", stream=None, split_k=True):
    M = A.shape[1] if transA else A.shape[0]
    K = A.shape[0] if transA else A.shape[1]
    N = B.shape[0] if transB else B.shape[1]
    C = torch.empty((M, N), dtype=A.dtype, device=A.device)
    wb = lib().ctm_debug_gemm_work_bytes(PREC[prec], M, N, K) if split_k else 0
    work = torch.empty(max(wb, 1), dtype=torch.uint8, device=A.device) if wb else None
    st = lib().ctm_debug_gemm(PREC[prec], int(transA), int(transB), M, N, K, _ptr(A.contiguous()),
                              _ptr(B.contiguous()), _ptr(C), _ptr(work) if work is not None else None,
                              _stream_ptr(torch, stream))
    if st != CTM_OK:
        raise CtmError(st, "ctm_debug_gemm")
    return C


def debug_svd(M, stream=None, max_sweeps=0):
    if M.dim() == 2:
        M = M[None]
    b, n, _ = M.shape
    M = M.contiguous()
    U = torch.empty_like(M)
    V = torch.empty_like(M)
    S = torch.empty((b, n), dtype=torch.float64, device=M.device)
    work = torch.empty(lib().ctm_debug_svd_work_bytes(n, b), dtype=torch.uint8, device=M.device)
    sw = ctypes.c_int(max_sweeps)
    st = lib().ctm_debug_svd(n, b, _ptr(M), _ptr(U), _ptr(S), _ptr(V), _ptr(work), ctypes.byref(sw),
                             _stream_ptr(torch, stream))
    if st != CTM_OK:
        raise CtmError(st, "ctm_debug_svd")
    return U, S, V, sw.value


def debug_qr(X, stream=None):
    """Thin QR of a batch of tall matrices X [batch, m, k] (FP64, device):
    returns (Q [batch, m, k], R [batch, k, k])."""
    if X.dim() == 2:
        X = X[None]
    b, m, k = X.shape
    Xt = X.transpose(1, 2).contiguous()
    R = torch.empty((b, k, k), dtype=torch.float64, device=X.device)
    Qt = torch.empty((b, k, m), dtype=torch.float64, device=X.device)
    work = torch.empty(max(lib().ctm_debug_qr_work_bytes(m, k, b), 1), dtype=torch.uint8, device=X.device)
    st = lib().ctm_debug_qr(m, k, b, _ptr(Xt), _ptr(R), _ptr(Qt), _ptr(work), _stream_ptr(torch, stream))
    if st != CTM_OK:
        raise CtmError(st, "ctm_debug_qr")
    return Qt.transpose(1, 2), R


class CtmEnergy(torch.autograd.Function):
    """E(A) after a fixed number of split-CTMRG sweeps, with dE/dA from the
    library's hand-written adjoints (Sec. III: the gradient by reverse mode
    through the CTMRG).  Call it through `ctm_energy` (keyword arguments);
    the positional form is

        CtmEnergy.apply(A, h, chi_E, n_sweeps, ckpt_every, prec, chi_I, h_v,
                        alt_yr, half_teal, cutoff, state)

    A: FP64 device tensor [Lx, Ly, p, D, D, D, D]; h (h_v): FP64 host arrays
    p^2 x p^2, the horizontal (vertical) bond Hamiltonian; state: None, or a
    dict whose "env" entry (packed FP64 device environment) is the start
    environment of the sweeps and receives the environment after them, so
    that successive calls (an optimiser's steps) start from the last one.
    Each call builds its own context: the library copies A at init."""

    @staticmethod
    def forward(ctx, A, h, chi_E, n_sweeps, ckpt_every, prec, chi_I, h_v, alt_yr, half_teal, cutoff, state):
        obj = SplitCTM(A.detach(), chi_E, chi_I if chi_I is not None else chi_E, prec=prec, with_grad=True,
                       n_sweeps=n_sweeps, ckpt_every=ckpt_every, cutoff=cutoff, alt_yr=alt_yr,
                       half_teal=half_teal)
        try:
            if state is not None and state.get("env") is not None:
                obj.env_import(state["env"])
            e, dA = obj.energy_grad(h, n_sweeps, ckpt_every, h_v=h_v)
            if state is not None:
                state["env"] = obj.env_export()
        finally:
            obj.close()
        ctx.save_for_backward(dA)
        return torch.tensor(e, dtype=torch.float64, device=A.device)

    @staticmethod
    def backward(ctx, ge):
        (dA,) = ctx.saved_tensors
        return (ge * dA,) + (None,) * 11


def ctm_energy(A, h, chi_E, n_sweeps, ckpt_every=1, prec="fp64", chi_I=None, h_v=None, alt_yr=False,
               half_teal=False, cutoff=1e-12, state=None):
    """Differentiable energy per site E(A) (see CtmEnergy)."""
    return CtmEnergy.apply(A, h, chi_E, n_sweeps, ckpt_every, prec, chi_I, h_v, alt_yr, half_teal, cutoff, state)
