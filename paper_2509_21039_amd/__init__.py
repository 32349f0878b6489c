"""MI355X-native two-electron Fock build (screened unique ERIs over contracted s Gaussians).

A thin ctypes binding over ``libhfk.so`` (see ``include/hfk.h``): it marshals torch tensors
into device pointers and the current HIP stream, and every step of the computation runs
in the library's HIP kernels.  PyTorch provides device memory and streams only.  There is
no CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhfk.so")

HFK_OK, HFK_EINVAL, HFK_ENOMEM, HFK_EHIP, HFK_EUNSUPPORTED, HFK_ENOTSYM = 0, 1, 2, 3, 4, 5
FP64, MIXED = 0, 1
STRATEGY_AUTO, STRATEGY_PRIVATE, STRATEGY_ATOMIC, STRATEGY_DETERMINISTIC = 0, 1, 2, 3
MAX_NGAUSS = 8

_PREC = {"fp64": FP64, "mixed": MIXED, FP64: FP64, MIXED: MIXED}

_STATUS_NAMES = {HFK_OK: "HFK_OK", HFK_EINVAL: "HFK_EINVAL", HFK_ENOMEM: "HFK_ENOMEM",
                 HFK_EHIP: "HFK_EHIP", HFK_EUNSUPPORTED: "HFK_EUNSUPPORTED", HFK_ENOTSYM: "HFK_ENOTSYM"}


class HfkError(RuntimeError):
    """A non-OK hfk_status, with the library's message."""

    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (_STATUS_NAMES.get(status, str(status)), message))
        self.status = status
        self.message = message


class HfkStats(ctypes.Structure):
    _fields_ = [("natoms", ctypes.c_int64), ("pairs", ctypes.c_int64), ("sig_pairs", ctypes.c_int64),
                ("quartets", ctypes.c_int64), ("work_items", ctypes.c_int64),
                ("strategy", ctypes.c_int32), ("groups", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("tile_items", ctypes.c_int32), ("group_bras", ctypes.c_int32),
                ("ket_copies", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_vp, _dp, _i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)
_sz = ctypes.c_size_t

_SIGNATURES = {
    "hfk_workspace_bytes": [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_sz)],
    "hfk_fock": [ctypes.c_int64, _vp, ctypes.c_int32, _dp, _dp, _vp, ctypes.c_double, ctypes.c_int32,
                 ctypes.c_int32, _vp, _vp, _vp, _sz, _vp],
    "hfk_fock_grad": [ctypes.c_int64, _vp, ctypes.c_int32, _dp, _dp, _vp, ctypes.c_double, ctypes.c_int32,
                      _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp],
    "hfk_batched_workspace_bytes": [ctypes.c_int64, _i64p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.POINTER(_sz)],
    "hfk_fock_batched": [ctypes.c_int64, _i64p, _vp, ctypes.c_int32, _dp, _dp, _vp, ctypes.c_double,
                         ctypes.c_int32, _vp, _vp, _vp, _vp, _sz, _vp],
    "hfk_read_stats": [_vp, _vp, ctypes.POINTER(HfkStats)],
    "hfk_tune": [ctypes.c_int64, _vp, ctypes.c_int32, _dp, _dp, _vp, ctypes.c_double, ctypes.c_int32,
                 _vp, _vp, _vp, _sz, _vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)],
    "hfk_load_tuning": [ctypes.c_char_p],
    "hfk_tune_batched": [ctypes.c_int64, _i64p, _vp, ctypes.c_int32, _dp, _dp, _vp, ctypes.c_double,
                         ctypes.c_int32, _vp, _vp, _vp, _vp, _sz, _vp, ctypes.c_char_p,
                         ctypes.POINTER(ctypes.c_int32)],
    "hfk_profile_enable": [ctypes.c_int32],
    "hfk_set_config": [ctypes.c_int32, ctypes.c_int32],
    "hfk_set_shape": [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
    "hfk_set_batched_config": [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32],
    "hfk_set_debug": [ctypes.c_int32, ctypes.c_double],
    "hfk_last_stats": [ctypes.POINTER(HfkStats)],
    "hfk_clear_tuning": [],
    "hfk_profile_read": [ctypes.POINTER(ctypes.c_double), _i64p],
    "hfk_workspace_bytes_atoms": [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.POINTER(_sz)],
    "hfk_batched_workspace_bytes_atoms": [ctypes.c_int64, _i64p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(_sz)],
    "hfk_fock_batched_atoms": [ctypes.c_int64, _i64p, _vp, ctypes.c_int32, _dp, _dp, _vp, ctypes.c_double,
                               ctypes.c_int32, _vp, _vp, _vp, _vp, _sz, _vp],
    "hfk_scf_workspace_bytes": [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_sz)],
    "hfk_scf": [ctypes.c_int64, _vp, _dp, ctypes.c_int32, _dp, _dp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double, _vp, ctypes.c_int32, _vp,
                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                _vp, _sz, _vp],
    "hfk_fock_grad_atoms": [ctypes.c_int64, _vp, ctypes.c_int32, _dp, _dp, _vp, ctypes.c_double, ctypes.c_int32,
                            _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp],
    "hfk_fock_atoms": [ctypes.c_int64, _vp, ctypes.c_int32, _dp, _dp, _vp, ctypes.c_double, ctypes.c_int32,
                       ctypes.c_int32, _vp, _vp, _vp, _sz, _vp],
    "hfk_fock_noalloc": [ctypes.c_int64, _vp, ctypes.c_int32, _dp, _dp, _vp, ctypes.c_double, ctypes.c_int32,
                         _vp, _vp, _vp],
}


def lib():
    """The loaded libhfk.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise HfkError(HFK_EUNSUPPORTED, "libhfk.so is not built (run paper_2509_21039_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.hfk_last_error.restype = ctypes.c_char_p
        L.hfk_last_error.argtypes = []
        L.hfk_version.restype = ctypes.c_char_p
        L.hfk_version.argtypes = []
        _lib = L
    return _lib


def _check(status: int):
    if status != HFK_OK:
        raise HfkError(status, lib().hfk_last_error().decode())


def _host_f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_f64(t, name: str, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise HfkError(HFK_EINVAL, "%s must be a device tensor" % name)
    if t.dtype != torch.float64:
        raise HfkError(HFK_EINVAL, "%s must be float64" % name)
    if not t.is_contiguous():
        raise HfkError(HFK_EINVAL, "%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise HfkError(HFK_EINVAL, "%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return t


def version() -> str:
    return lib().hfk_version().decode()


def workspace_bytes(natoms: int, ngauss: int = 3, precision="fp64", with_grad: bool = False) -> int:
    out = _sz(0)
    _check(lib().hfk_workspace_bytes(int(natoms), int(ngauss), _PREC[precision], int(bool(with_grad)),
                                     ctypes.byref(out)))
    return out.value


def new_workspace(nbytes: int, device=None):
    torch = _torch()
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device or "cuda")


def fock(xyz, dens, exps: Sequence[float], coefs: Sequence[float], tau: float, precision="fp64",
         strategy: int = STRATEGY_AUTO, workspace=None, out=None, stream=None):
    """Two-electron Fock matrix G and energy E2 (device tensors) for one molecule."""
    torch = _torch()
    n = xyz.shape[0]
    _dev_f64(xyz, "xyz", (n, 3))
    _dev_f64(dens, "dens", (n, n))
    e = _host_f64(exps)
    c = _host_f64(coefs)
    if e.shape != c.shape or e.ndim != 1:
        raise HfkError(HFK_EINVAL, "exps and coefs must be 1-D of equal length")
    prec = _PREC[precision]
    if workspace is None:
        workspace = new_workspace(workspace_bytes(n, len(e), prec), xyz.device)
    if out is None:
        F = torch.empty((n, n), dtype=torch.float64, device=xyz.device)
        E2 = torch.empty((1,), dtype=torch.float64, device=xyz.device)
    else:
        F, E2 = out
    _check(lib().hfk_fock(n, xyz.data_ptr(), len(e), _dptr(e), _dptr(c), dens.data_ptr(), float(tau), prec,
                          int(strategy), F.data_ptr(), E2.data_ptr(), workspace.data_ptr(),
                          workspace.numel(), _stream_handle(stream)))
    return F, E2


def fock_noalloc(xyz, dens, exps: Sequence[float], coefs: Sequence[float], tau: float, precision="fp64",
                 out=None, stream=None):
    """hfk_fock_noalloc: the forward build with the library's static scratch (no workspace);
    `out` = (F, E2) preallocated by the caller, or None to allocate them here."""
    torch = _torch()
    n = xyz.shape[0]
    _dev_f64(xyz, "xyz", (n, 3))
    _dev_f64(dens, "dens", (n, n))
    e = _host_f64(exps)
    c = _host_f64(coefs)
    if e.shape != c.shape or e.ndim != 1:
        raise HfkError(HFK_EINVAL, "exps and coefs must be 1-D of equal length")
    if out is None:
        F = torch.empty((n, n), dtype=torch.float64, device=xyz.device)
        E2 = torch.empty((1,), dtype=torch.float64, device=xyz.device)
    else:
        F, E2 = out
    _check(lib().hfk_fock_noalloc(n, xyz.data_ptr(), len(e), _dptr(e), _dptr(c), dens.data_ptr(), float(tau),
                                  _PREC[precision], F.data_ptr(), E2.data_ptr(), _stream_handle(stream)))
    return F, E2


def workspace_bytes_atoms(natoms: int, ngauss: int = 3, precision="fp64", with_grad: bool = False) -> int:
    out = _sz(0)
    _check(lib().hfk_workspace_bytes_atoms(int(natoms), int(ngauss), _PREC[precision], int(bool(with_grad)),
                                           ctypes.byref(out)))
    return out.value


def _rows(exps, coefs, n):
    e = _host_f64(exps)
    c = _host_f64(coefs)
    if e.shape != c.shape or e.ndim != 2 or e.shape[0] != n:
        raise HfkError(HFK_EINVAL, "per-atom exps and coefs must both be (natoms, ngauss)")
    return e, c


def fock_atoms(xyz, dens, exps, coefs, tau: float, precision="fp64", strategy: int = STRATEGY_AUTO,
               workspace=None, out=None, stream=None):
    """G and E2 with per-atom bases: exps and coefs are (natoms, ngauss) host arrays, row i the
    contraction of atom i."""
    torch = _torch()
    n = xyz.shape[0]
    _dev_f64(xyz, "xyz", (n, 3))
    _dev_f64(dens, "dens", (n, n))
    e, c = _rows(exps, coefs, n)
    g = e.shape[1]
    prec = _PREC[precision]
    if workspace is None:
        workspace = new_workspace(workspace_bytes_atoms(n, g, prec), xyz.device)
    if out is None:
        F = torch.empty((n, n), dtype=torch.float64, device=xyz.device)
        E2 = torch.empty((1,), dtype=torch.float64, device=xyz.device)
    else:
        F, E2 = out
    _check(lib().hfk_fock_atoms(n, xyz.data_ptr(), g, _dptr(e), _dptr(c), dens.data_ptr(), float(tau), prec,
                                int(strategy), F.data_ptr(), E2.data_ptr(), workspace.data_ptr(),
                                workspace.numel(), _stream_handle(stream)))
    return F, E2


def scf_workspace_bytes(natoms: int, ngauss: int = 3, precision="fp64") -> int:
    out = _sz(0)
    _check(lib().hfk_scf_workspace_bytes(int(natoms), int(ngauss), _PREC[precision], ctypes.byref(out)))
    return out.value


def scf(xyz, charges, exps, coefs, nocc: int, tau: float, precision="fp64", strategy: int = STRATEGY_AUTO,
        max_iter: int = 100, e_tol: float = 1e-10, d_tol: float = 1e-7, dens0=None, workspace=None, stream=None):
    """Closed-shell SCF around the two-electron build.  charges: (natoms,) nuclear charges
    (host); exps/coefs: per-atom rows (natoms, ngauss); dens0: optional device (n, n) start.
    Returns dict(E, D (device), eps (device), iterations, converged)."""
    torch = _torch()
    n = xyz.shape[0]
    _dev_f64(xyz, "xyz", (n, 3))
    e, c = _rows(exps, coefs, n)
    g = e.shape[1]
    Z = _host_f64(charges)
    if Z.shape != (n,):
        raise HfkError(HFK_EINVAL, "charges must be (natoms,)")
    prec = _PREC[precision]
    if workspace is None:
        workspace = new_workspace(scf_workspace_bytes(n, g, prec), xyz.device)
    if dens0 is not None:
        _dev_f64(dens0, "dens0", (n, n))
        D = dens0.clone()
    else:
        D = torch.empty((n, n), dtype=torch.float64, device=xyz.device)
    eps = torch.empty((n,), dtype=torch.float64, device=xyz.device)
    E = ctypes.c_double(0.0)
    its = ctypes.c_int32(0)
    conv = ctypes.c_int32(0)
    _check(lib().hfk_scf(n, xyz.data_ptr(), _dptr(Z), g, _dptr(e), _dptr(c), int(nocc), float(tau), prec,
                         int(strategy), int(max_iter), float(e_tol), float(d_tol), D.data_ptr(),
                         int(dens0 is not None), eps.data_ptr(), ctypes.byref(E), ctypes.byref(its),
                         ctypes.byref(conv), workspace.data_ptr(), workspace.numel(), _stream_handle(stream)))
    return {"E": E.value, "D": D, "eps": eps, "iterations": its.value, "converged": bool(conv.value)}


def read_stats(workspace, stream=None) -> dict:
    st = HfkStats()
    _check(lib().hfk_read_stats(workspace.data_ptr(), _stream_handle(stream), ctypes.byref(st)))
    return st.as_dict()


def fock_grad(xyz, dens, exps, coefs, tau, precision="fp64", g_e2=None, fock_in=None, want_dens=True,
              workspace=None, stream=None, g_fock=None):
    """(d_xyz, d_dens or None, E2) for upstream g_e2 (device scalar tensor; 1 if None) and
    g_fock (device [n, n] tensor dL/dG, or None).  exps/coefs: one contraction (1-D) for every
    atom, or per-atom rows (natoms, ngauss)."""
    torch = _torch()
    n = xyz.shape[0]
    _dev_f64(xyz, "xyz", (n, 3))
    _dev_f64(dens, "dens", (n, n))
    atoms = np.ndim(exps) == 2
    if atoms:
        e, c = _rows(exps, coefs, n)
        g = e.shape[1]
    else:
        e = _host_f64(exps)
        c = _host_f64(coefs)
        g = len(e)
    prec = _PREC[precision]
    if g_e2 is None:
        g_e2 = torch.ones((1,), dtype=torch.float64, device=xyz.device)
    _dev_f64(g_e2, "g_e2")
    if workspace is None:
        nb = workspace_bytes_atoms(n, g, prec, True) if atoms else workspace_bytes(n, g, prec, True)
        workspace = new_workspace(nb, xyz.device)
    if g_fock is not None:
        _dev_f64(g_fock, "g_fock", (n, n))
    d_xyz = torch.empty((n, 3), dtype=torch.float64, device=xyz.device)
    d_dens = None
    if want_dens:
        if fock_in is None:
            raise HfkError(HFK_EINVAL, "d_dens needs fock_in (G from the forward call)")
        _dev_f64(fock_in, "fock_in", (n, n))
        d_dens = torch.empty((n, n), dtype=torch.float64, device=xyz.device)
    E2 = torch.empty((1,), dtype=torch.float64, device=xyz.device)
    call = lib().hfk_fock_grad_atoms if atoms else lib().hfk_fock_grad
    _check(call(n, xyz.data_ptr(), g, _dptr(e), _dptr(c), dens.data_ptr(), float(tau), prec,
                g_e2.data_ptr(), g_fock.data_ptr() if g_fock is not None else None,
                fock_in.data_ptr() if fock_in is not None else None,
                d_xyz.data_ptr(), d_dens.data_ptr() if d_dens is not None else None,
                E2.data_ptr(), workspace.data_ptr(), workspace.numel(), _stream_handle(stream)))
    return d_xyz, d_dens, E2


def _autograd():
    torch = _torch()

    class FockEnergy(torch.autograd.Function):
        """E2 (and G) as a differentiable function of positions and density.

        forward(xyz, dens, exps, coefs, tau, precision) -> (G, E2); backward hands the
        upstream (gG, gE2) to the library's gradient call: dL/dxyz from the two-density
        contraction, dL/ddens = gE2 * G + G(sym(gG)).  exps/coefs: one contraction (1-D) or
        per-atom rows (natoms, ngauss)."""

        @staticmethod
        def forward(ctx, xyz, dens, exps, coefs, tau, precision="fp64"):
            ctx.set_materialize_grads(False)
            if np.ndim(exps) == 2:
                G, E2 = fock_atoms(xyz, dens, exps, coefs, tau, precision)
            else:
                G, E2 = fock(xyz, dens, exps, coefs, tau, precision)
            ctx.save_for_backward(xyz, dens, G)
            ctx.basis = (np.asarray(exps, dtype=np.float64).copy(), np.asarray(coefs, dtype=np.float64).copy())
            ctx.tau = tau
            ctx.precision = precision
            return G, E2

        @staticmethod
        def backward(ctx, gG, gE2):
            xyz, dens, G = ctx.saved_tensors
            if gE2 is None and gG is None:
                return None, None, None, None, None, None
            if gE2 is None:
                gE2 = torch.zeros((1,), dtype=torch.float64, device=xyz.device)
            e, c = ctx.basis
            d_xyz, d_dens, _ = fock_grad(xyz, dens, e, c, ctx.tau, ctx.precision,
                                         g_e2=gE2.reshape(1).to(torch.float64).contiguous(), fock_in=G,
                                         want_dens=ctx.needs_input_grad[1],
                                         g_fock=None if gG is None else gG.to(torch.float64).contiguous())
            return (d_xyz if ctx.needs_input_grad[0] else None, d_dens, None, None, None, None)

    return FockEnergy


_FockEnergy = None


def __getattr__(name):
    global _FockEnergy
    if name == "FockEnergy":
        if _FockEnergy is None:
            _FockEnergy = _autograd()
        return _FockEnergy
    raise AttributeError(name)


def batched_workspace_bytes(atom_off, ngauss=3, precision="mixed", with_grad=True, atoms=False) -> int:
    off = np.ascontiguousarray(np.asarray(atom_off, dtype=np.int64))
    out = _sz(0)
    call = lib().hfk_batched_workspace_bytes_atoms if atoms else lib().hfk_batched_workspace_bytes
    _check(call(len(off) - 1, off.ctypes.data_as(_i64p), int(ngauss), _PREC[precision], int(bool(with_grad)),
                ctypes.byref(out)))
    return out.value


def fock_batched(atom_off, xyz, dens_packed, exps, coefs, tau, precision="mixed", with_grad=True,
                 workspace=None, stream=None):
    """Ragged batch in one persistent launch: (fock_packed, e2[nmol], d_xyz or None).  exps/coefs:
    one contraction (1-D) for every atom, or per-atom rows (sum n, ngauss) over the stacked atoms."""
    torch = _torch()
    off = np.ascontiguousarray(np.asarray(atom_off, dtype=np.int64))
    nmol = len(off) - 1
    _dev_f64(xyz, "xyz", (int(off[-1]), 3))
    _dev_f64(dens_packed, "dens_packed")
    atoms = np.ndim(exps) == 2
    if atoms:
        e, c = _rows(exps, coefs, int(off[-1]))
        g = e.shape[1]
    else:
        e = _host_f64(exps)
        c = _host_f64(coefs)
        g = len(e)
    prec = _PREC[precision]
    if workspace is None:
        workspace = new_workspace(batched_workspace_bytes(off, g, prec, with_grad, atoms), xyz.device)
    F = torch.empty_like(dens_packed)
    E2 = torch.empty((nmol,), dtype=torch.float64, device=xyz.device)
    d_xyz = torch.empty_like(xyz) if with_grad else None
    call = lib().hfk_fock_batched_atoms if atoms else lib().hfk_fock_batched
    _check(call(nmol, off.ctypes.data_as(_i64p), xyz.data_ptr(), g, _dptr(e), _dptr(c),
                dens_packed.data_ptr(), float(tau), prec, F.data_ptr(), E2.data_ptr(),
                d_xyz.data_ptr() if d_xyz is not None else None, workspace.data_ptr(),
                workspace.numel(), _stream_handle(stream)))
    return F, E2, d_xyz


def tune(xyz, dens, exps, coefs, tau, precision="fp64", cache_path: Optional[str] = None, stream=None) -> int:
    """Runs the autotuner on this system; returns the chosen strategy."""
    torch = _torch()
    n = xyz.shape[0]
    e = _host_f64(exps)
    c = _host_f64(coefs)
    prec = _PREC[precision]
    ws = new_workspace(workspace_bytes(n, len(e), prec), xyz.device)
    F = torch.empty((n, n), dtype=torch.float64, device=xyz.device)
    E2 = torch.empty((1,), dtype=torch.float64, device=xyz.device)
    best = ctypes.c_int32(0)
    _check(lib().hfk_tune(n, xyz.data_ptr(), len(e), _dptr(e), _dptr(c), dens.data_ptr(), float(tau), prec,
                          F.data_ptr(), E2.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(stream),
                          cache_path.encode() if cache_path else None, ctypes.byref(best)))
    return best.value


def set_config(variant: int = -1, groups_per_cu: int = 0):
    """Override the quartet-kernel variant (0 direct, 1 near/far split, -1 library choice)
    and the persistent workgroups per compute unit (0 = default), process-wide."""
    _check(lib().hfk_set_config(int(variant), int(groups_per_cu)))


def profile_enable(on: bool = True):
    """Record HIP events around every quartet-kernel launch (measurement tools only)."""
    _check(lib().hfk_profile_enable(int(bool(on))))


def profile_read():
    """(summed quartet-kernel milliseconds, launches) since the last read; waits for them."""
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    _check(lib().hfk_profile_read(ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


def tune_batched(atom_off, xyz, dens_packed, exps, coefs, tau, precision="mixed", with_grad=True,
                 cache_path: Optional[str] = None, stream=None) -> int:
    """Runs the batched autotuner; returns the chosen workgroups per compute unit."""
    torch = _torch()
    off = np.ascontiguousarray(np.asarray(atom_off, dtype=np.int64))
    nmol = len(off) - 1
    e = _host_f64(exps)
    c = _host_f64(coefs)
    prec = _PREC[precision]
    ws = new_workspace(batched_workspace_bytes(off, len(e), prec, with_grad), xyz.device)
    F = torch.empty_like(dens_packed)
    E2 = torch.empty((nmol,), dtype=torch.float64, device=xyz.device)
    g = torch.empty_like(xyz) if with_grad else None
    best = ctypes.c_int32(0)
    _check(lib().hfk_tune_batched(nmol, off.ctypes.data_as(_i64p), xyz.data_ptr(), len(e), _dptr(e), _dptr(c),
                                  dens_packed.data_ptr(), float(tau), prec, F.data_ptr(), E2.data_ptr(),
                                  g.data_ptr() if g is not None else None, ws.data_ptr(), ws.numel(),
                                  _stream_handle(stream), cache_path.encode() if cache_path else None,
                                  ctypes.byref(best)))
    return best.value


def load_tuning(cache_path: str):
    _check(lib().hfk_load_tuning(cache_path.encode()))


def clear_tuning():
    """Forget every tuned configuration of the process (hfk_clear_tuning)."""
    _check(lib().hfk_clear_tuning())


def set_shape(tile_items: int = 0, group_bras: int = 0, ket_copies: int = -1):
    """Override the quartet-tile shape (hfk_set_shape); the defaults restore the library's choice."""
    _check(lib().hfk_set_shape(int(tile_items), int(group_bras), int(ket_copies)))


def set_batched_config(groups_per_cu: int = 0, block_items: int = 0, owned_bound: int = 0, waves: int = 0):
    """Override the batched launch (hfk_set_batched_config); the defaults restore the library's choice."""
    _check(lib().hfk_set_batched_config(int(groups_per_cu), int(block_items), int(owned_bound), int(waves)))


def set_debug(on: bool = True, sym_tol: float = 0.0):
    """Debug mode (hfk_set_debug): densities are checked on the device before every build."""
    _check(lib().hfk_set_debug(1 if on else 0, float(sym_tol)))


def last_stats() -> dict:
    """Counters of this thread's last build call (hfk_last_stats; waits for its stream)."""
    st = HfkStats()
    _check(lib().hfk_last_stats(ctypes.byref(st)))
    return st.as_dict()
