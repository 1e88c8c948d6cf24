"""Python binding of libqm_hpsi (MI355X / gfx950 plane-wave H|psi> and block Davidson).

Thin ctypes layer over the C ABI declared in include/qm_hpsi.h: every function
here has the name of the C entry point it calls and only marshals arguments
(torch tensors -> device pointers, numpy arrays -> host pointers, the current
torch stream -> hipStream_t).  All arithmetic runs in the HIP library; if the
library is not built, every call raises.

Physics: the Kohn-Sham Hamiltonian of the plane-wave basis at a k-point
(kinetic, local potential via FFT, Kleinman-Bylander projectors; paper
Secs. 2.2, 2.3, 4.3) and the block Davidson eigensolver built on it (Sec. 5).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqm_hpsi.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "qm_hpsi.h")

QM_OK, QM_E_ARG, QM_E_SHAPE, QM_E_HIP, QM_E_NOMEM, QM_E_NOT_SPD, QM_E_NOT_CONVERGED, QM_E_NAN, \
    QM_E_STATE = range(9)
QM_PREC_FP64, QM_PREC_FP32, QM_PREC_MIXED = 0, 1, 2
QM_PRECOND_TETER, QM_PRECOND_MLP = 0, 1
QM_MLP_NIN, QM_MLP_NHID = 5, 128
QM_MLP_NPARAM = 128 * 5 + 128 + 2 * 128 + 2

_STATUS = {0: "QM_OK", 1: "QM_E_ARG", 2: "QM_E_SHAPE", 3: "QM_E_HIP", 4: "QM_E_NOMEM",
           5: "QM_E_NOT_SPD", 6: "QM_E_NOT_CONVERGED", 7: "QM_E_NAN", 8: "QM_E_STATE"}


class QmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class qm_kset(ctypes.Structure):
    _fields_ = [("nk", ctypes.c_int32), ("k_cart", ctypes.c_void_p),
                ("npw", ctypes.c_void_p), ("miller", ctypes.c_void_p)]


class qm_dav_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("max_basis", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("restart", ctypes.c_int32), ("switch_resid", ctypes.c_double),
                ("mlp_weights", ctypes.c_void_p), ("lanes", ctypes.c_int32),
                ("extra_bands", ctypes.c_int32), ("subspace_fp32", ctypes.c_int32)]


class qm_scf_opts(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("dav", qm_dav_opts)]


class qm_scf_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("dav_iterations", ctypes.c_int64), ("n_hpsi_bands", ctypes.c_int64),
                ("residual", ctypes.c_double), ("e_hartree", ctypes.c_double),
                ("t_total_ms", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class qm_dav_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("n_hpsi_bands", ctypes.c_int64), ("n_hpsi_bands_lowp", ctypes.c_int64),
                ("max_resnorm", ctypes.c_double), ("t_hpsi_ms", ctypes.c_double),
                ("t_subspace_ms", ctypes.c_double), ("t_eig_ms", ctypes.c_double),
                ("t_total_ms", ctypes.c_double), ("n_gs", ctypes.c_int64),
                ("n_gs_second", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_LIB = None
_P = ctypes.c_void_p


def _load():
    global _LIB
    if _LIB is not None:
        return _LIB
    import torch  # noqa: F401  (the library binds to the HIP runtime torch has loaded)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2308_07277_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, dbl, flt = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_float
    sig = {
        "qm_hpsi_plan_create": [_P, _P, ctypes.POINTER(qm_kset), i32, i32, _P, _P, _P, i32, _P,
                                ctypes.POINTER(_P)],
        "qm_hpsi_plan_destroy": [_P],
        "qm_hpsi_plan_set_precision": [_P, i32, _P],
        "qm_hpsi_plan_set_graphs": [_P, i32],
        "qm_hpsi_plan_autotune": [_P, i32, _P],
        "qm_apply_h": [_P, i32, _P, _P, i32, _P],
        "qm_apply_h_timed": [_P, i32, _P, _P, i32, _P, _P],
        "qm_apply_h_noalloc": [_P, i32, _P, _P, i32, _P],
        "qm_davidson_step": [_P, i32, _P, _P, _P, i32, ctypes.POINTER(qm_dav_opts), _P, _P],
        "qm_davidson_solve": [_P, i32, _P, _P, _P, i32, ctypes.POINTER(qm_dav_opts),
                              ctypes.POINTER(qm_dav_stats), _P],
        "qm_mlp_forward": [_P, _P, _P, i64, _P],
        "qm_mlp_loss_grad": [_P, _P, _P, _P, _P, i32, _P, _P, _P],
        "qm_dav_training_pairs": [_P, _P, _P, dbl, _P, _P, _P, _P, i64, i32, _P, _P, _P],
        "qm_mlp_adam": [_P, _P, _P, _P, i32, flt, flt, flt, flt, _P],
        "qm_density": [_P, i32, _P, i32, _P, _P, _P, _P],
        "qm_hartree": [_P, _P, _P, _P, _P],
        "qm_hpsi_plan_set_vloc": [_P, _P, _P],
        "qm_scf_hartree": [_P, _P, _P, i32, _P, i32, ctypes.POINTER(qm_scf_opts), _P, _P, _P,
                           ctypes.POINTER(qm_scf_stats), _P],
        "qm_expm_taylor": [_P, i32, _P, _P, i32, dbl, i32, _P],
        "qm_td_etrs": [_P, _P, _P, _P, _P, i32, dbl, i32, i32, _P],
        "qm_mtxel": [_P, i32, _P, i32, i32, _P, i32, _P, i32, _P, _P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = None if name == "qm_hpsi_plan_destroy" else ctypes.c_int
    lib.qm_last_error.argtypes = [_P]
    lib.qm_last_error.restype = ctypes.c_char_p
    _LIB = lib
    return lib


def lib_loaded_path():
    _load()
    return LIB_PATH


def _stream(stream):
    import torch
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _dev(t, dtype=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP torch tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _check(status, handle=None):
    if status != QM_OK:
        msg = _load().qm_last_error(handle).decode(errors="replace")
        raise QmError(status, msg)


class HpsiPlan:
    """Owns a qm_hpsi_plan handle; destroyed with the object or by close()."""

    def __init__(self, handle, nk, npw, nbnd_max, nproj, grid):
        self.handle = handle
        self.nk = nk
        self.npw = np.asarray(npw, np.int64)
        self.nbnd_max = nbnd_max
        self.nproj = nproj
        self.grid = tuple(grid)

    def close(self):
        if self.handle:
            _load().qm_hpsi_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def band_block_numel(self, nbnd, k=-1):
        """Elements of a [(nk,) nbnd, npw_k] block, or None when k is not a valid index
        (the library itself then reports QM_E_ARG)."""
        if k < -1 or k >= self.nk:
            return None
        return int(nbnd * (self.npw.sum() if k < 0 else self.npw[k]))


def qm_hpsi_plan_create(cell, grid, k_cart, npw, miller, nbnd_max, nproj, vloc_r, beta, dmat,
                        prec=QM_PREC_FP64, stream=None):
    """cell [3,3] bohr (rows a_i); grid (N1,N2,N3); k_cart [nk,3] bohr^-1; npw [nk];
    miller int [sum npw, 3]; vloc_r torch float64 device [N1,N2,N3]; beta torch complex128
    device [sum_k nproj*npw_k] (k blocks of [nproj][npw_k]) or None; dmat [nproj,nproj]."""
    import torch
    lib = _load()
    cell = np.ascontiguousarray(cell, np.float64).reshape(9)
    grid_a = np.ascontiguousarray(grid, np.int32).reshape(3)
    k_cart = np.ascontiguousarray(k_cart, np.float64).reshape(-1, 3)
    npw = np.ascontiguousarray(npw, np.int32).reshape(-1)
    miller = np.ascontiguousarray(miller, np.int32).reshape(-1, 3)
    if k_cart.shape[0] != npw.shape[0] or miller.shape[0] != int(npw.sum()):
        raise ValueError("k_cart, npw and miller disagree in size")
    ks = qm_kset(int(npw.shape[0]), k_cart.ctypes.data, npw.ctypes.data, miller.ctypes.data)
    vp = _dev(vloc_r, torch.float64, "vloc_r")
    if nproj > 0:
        bp = _dev(beta, torch.complex128, "beta")
        dm = np.ascontiguousarray(dmat, np.float64).reshape(nproj, nproj)
        dp = ctypes.c_void_p(dm.ctypes.data)
    else:
        bp, dp, dm = ctypes.c_void_p(0), ctypes.c_void_p(0), None
    out = ctypes.c_void_p(0)
    st = lib.qm_hpsi_plan_create(cell.ctypes.data, grid_a.ctypes.data, ctypes.byref(ks),
                                 int(nbnd_max), int(nproj), vp, bp, dp, int(prec),
                                 _stream(stream), ctypes.byref(out))
    _check(st, None)
    return HpsiPlan(out, int(npw.shape[0]), npw, int(nbnd_max), int(nproj), grid_a)


def qm_hpsi_plan_set_precision(plan, prec, stream=None):
    _check(_load().qm_hpsi_plan_set_precision(plan.handle, int(prec), _stream(stream)), plan.handle)


def qm_hpsi_plan_autotune(plan, nbnd, stream=None):
    _check(_load().qm_hpsi_plan_autotune(plan.handle, int(nbnd), _stream(stream)), plan.handle)


def qm_hpsi_plan_set_graphs(plan, enable):
    _check(_load().qm_hpsi_plan_set_graphs(plan.handle, int(bool(enable))), plan.handle)


def qm_apply_h(plan, k, psi, hpsi, nbnd, stream=None):
    """hpsi <- H(k) psi; psi/hpsi complex128 device tensors [(nk,) nbnd, npw_k] (k=-1: all k)."""
    import torch
    n = plan.band_block_numel(nbnd, k)
    if n is not None and (psi.numel() != n or hpsi.numel() != n):
        raise ValueError(f"psi/hpsi must hold {n} elements for nbnd={nbnd}, k={k}")
    _check(_load().qm_apply_h(plan.handle, int(k), _dev(psi, torch.complex128, "psi"),
                              _dev(hpsi, torch.complex128, "hpsi"), int(nbnd), _stream(stream)),
           plan.handle)


def qm_apply_h_noalloc(plan, k, psi, hpsi, nbnd, stream=None):
    """qm_apply_h without any device allocation (working memory in the library's static
    scratch array); same arguments and results."""
    import torch
    n = plan.band_block_numel(nbnd, k)
    if n is not None and (psi.numel() != n or hpsi.numel() != n):
        raise ValueError(f"psi/hpsi must hold {n} elements for nbnd={nbnd}, k={k}")
    _check(_load().qm_apply_h_noalloc(plan.handle, int(k), _dev(psi, torch.complex128, "psi"),
                                      _dev(hpsi, torch.complex128, "hpsi"), int(nbnd),
                                      _stream(stream)), plan.handle)


QM_NSTAGES = 7
STAGE_NAMES = ("zinv", "xy", "zfwd", "proj_gemm", "proj_reduce", "apply_d", "expand_gemm")


def qm_apply_h_timed(plan, k, psi, hpsi, nbnd, stream=None):
    """qm_apply_h with per-stage HIP-event timings; returns a dict stage -> ms."""
    import torch
    n = plan.band_block_numel(nbnd, k)
    if n is not None and (psi.numel() != n or hpsi.numel() != n):
        raise ValueError(f"psi/hpsi must hold {n} elements for nbnd={nbnd}, k={k}")
    t = np.zeros(QM_NSTAGES)
    _check(_load().qm_apply_h_timed(plan.handle, int(k), _dev(psi, torch.complex128, "psi"),
                                    _dev(hpsi, torch.complex128, "hpsi"), int(nbnd),
                                    t.ctypes.data, _stream(stream)), plan.handle)
    return dict(zip(STAGE_NAMES, t.tolist()))


def _opts(tol=1e-8, max_iter=200, max_basis=0, precond=QM_PRECOND_TETER, restart=0,
          switch_resid=0.0, mlp_weights=None, lanes=0, extra_bands=0, subspace_fp32=0):
    w = 0 if mlp_weights is None else mlp_weights.data_ptr()
    return qm_dav_opts(float(tol), int(max_iter), int(max_basis), int(precond), int(restart),
                       float(switch_resid), ctypes.c_void_p(w), int(lanes), int(extra_bands),
                       int(subspace_fp32))


def qm_davidson_step(plan, k, psi, nbnd, stream=None, **opts):
    """One Davidson iteration; returns (eig [nk_sel, nbnd], resnorm [nk_sel, nbnd], n_unconverged)."""
    import torch
    nks = plan.nk if k < 0 else 1
    eig = np.zeros((nks, nbnd))
    res = np.zeros((nks, nbnd))
    nun = ctypes.c_int32(0)
    o = _opts(**opts)
    _check(_load().qm_davidson_step(plan.handle, int(k), _dev(psi, torch.complex128, "psi"),
                                    eig.ctypes.data, res.ctypes.data, int(nbnd), ctypes.byref(o),
                                    ctypes.byref(nun), _stream(stream)), plan.handle)
    return eig, res, int(nun.value)


def qm_davidson_solve(plan, k, psi, nbnd, stream=None, raise_not_converged=False, **opts):
    """Davidson to convergence; psi (in: start, out: Ritz vectors).
    Returns (eig, resnorm, stats dict, status)."""
    import torch
    nks = plan.nk if k < 0 else 1
    eig = np.zeros((nks, nbnd))
    res = np.zeros((nks, nbnd))
    stats = qm_dav_stats()
    o = _opts(**opts)
    st = _load().qm_davidson_solve(plan.handle, int(k), _dev(psi, torch.complex128, "psi"),
                                   eig.ctypes.data, res.ctypes.data, int(nbnd), ctypes.byref(o),
                                   ctypes.byref(stats), _stream(stream))
    if st != QM_OK and (st != QM_E_NOT_CONVERGED or raise_not_converged):
        _check(st, plan.handle)
    return eig, res, stats.as_dict(), st


def qm_mlp_forward(weights, feat, gain, n, stream=None):
    import torch
    _check(_load().qm_mlp_forward(_dev(weights, torch.float32, "weights"),
                                  _dev(feat, torch.float32, "feat"),
                                  _dev(gain, torch.float32, "gain"), int(n), _stream(stream)))


def qm_mlp_loss_grad(weights, feat, resid, target, band_ptr, nbands, grad, stream=None):
    """Per-band cosine loss and its gradient (device tensors); returns the loss."""
    import torch
    loss = ctypes.c_double(0.0)
    _check(_load().qm_mlp_loss_grad(_dev(weights, torch.float32, "weights"),
                                    _dev(feat, torch.float32, "feat"),
                                    _dev(resid, torch.float32, "resid"),
                                    _dev(target, torch.float32, "target"),
                                    _dev(band_ptr, torch.int32, "band_ptr"), int(nbands),
                                    _dev(grad, torch.float32, "grad"), ctypes.byref(loss),
                                    _stream(stream)))
    return loss.value


def qm_dav_training_pairs(plan, x_star, eig_star, feat, resid, target, band_ptr, cluster_tol=0.0,
                          stream=None):
    """Training rows from the plan's current Davidson state; returns (nrows, nbands)."""
    import torch
    es = np.ascontiguousarray(eig_star, np.float64)
    nrows = ctypes.c_int64(0)
    nb = ctypes.c_int32(0)
    _check(_load().qm_dav_training_pairs(plan.handle, _dev(x_star, torch.complex128, "x_star"),
                                         es.ctypes.data, float(cluster_tol),
                                         _dev(feat, torch.float32, "feat"),
                                         _dev(resid, torch.float32, "resid"),
                                         _dev(target, torch.float32, "target"),
                                         _dev(band_ptr, torch.int32, "band_ptr"),
                                         int(feat.shape[0]), int(band_ptr.numel()) - 1,
                                         ctypes.byref(nrows), ctypes.byref(nb), _stream(stream)),
           plan.handle)
    return int(nrows.value), int(nb.value)


def qm_mlp_adam(weights, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    import torch
    _check(_load().qm_mlp_adam(_dev(weights, torch.float32, "weights"),
                               _dev(grad, torch.float32, "grad"), _dev(m, torch.float32, "m"),
                               _dev(v, torch.float32, "v"), int(t), float(lr), float(beta1),
                               float(beta2), float(eps), _stream(stream)))


def qm_density(plan, k, psi, nbnd, weights, occ, rho, stream=None):
    """rho <- sum_k w_k sum_n f_kn |psi_kn(r)|^2 on the plan's grid (float64 device tensor
    [N1, N2, N3]); weights [nk_sel], occ [nk_sel, nbnd] host arrays."""
    import torch
    nks = plan.nk if k < 0 else 1
    w = np.ascontiguousarray(weights, np.float64).reshape(-1)
    f = np.ascontiguousarray(occ, np.float64).reshape(-1)
    if w.size != nks or f.size != nks * nbnd:
        raise ValueError("weights must hold nk_sel values and occ nk_sel * nbnd")
    n = plan.band_block_numel(nbnd, k)
    if n is not None and psi.numel() != n:
        raise ValueError(f"psi must hold {n} elements")
    if rho.numel() != int(np.prod(plan.grid)):
        raise ValueError("rho must hold N1*N2*N3 values")
    _check(_load().qm_density(plan.handle, int(k), _dev(psi, torch.complex128, "psi"), int(nbnd),
                              w.ctypes.data, f.ctypes.data, _dev(rho, torch.float64, "rho"),
                              _stream(stream)), plan.handle)


def qm_hartree(plan, rho, vh, energy=False, stream=None):
    """vh <- Hartree potential of rho (float64 device grids); returns E_H if energy."""
    import torch
    for t, nm in ((rho, "rho"), (vh, "vh")):
        if t.numel() != int(np.prod(plan.grid)):
            raise ValueError(f"{nm} must hold N1*N2*N3 values")
    e = ctypes.c_double(0.0)
    _check(_load().qm_hartree(plan.handle, _dev(rho, torch.float64, "rho"), _dev(vh, torch.float64, "vh"),
                              ctypes.byref(e) if energy else None, _stream(stream)), plan.handle)
    return e.value if energy else None


def qm_hpsi_plan_set_vloc(plan, vloc_r, stream=None):
    import torch
    if vloc_r.numel() != int(np.prod(plan.grid)):
        raise ValueError("vloc_r must hold N1*N2*N3 values")
    _check(_load().qm_hpsi_plan_set_vloc(plan.handle, _dev(vloc_r, torch.float64, "vloc_r"),
                                         _stream(stream)), plan.handle)


def qm_scf_hartree(plan, vext, kweights, nocc, psi, nbnd, rho, vh, alpha=0.0, tol=0.0, max_iter=0,
                   stream=None, **dav_opts):
    """Hartree-only SCF; returns (eig [nk, nbnd], stats dict, status)."""
    import torch
    kw = np.ascontiguousarray(kweights, np.float64).reshape(-1)
    if kw.size != plan.nk:
        raise ValueError("kweights must hold nk values")
    n = plan.band_block_numel(nbnd, -1)
    if psi.numel() != n:
        raise ValueError(f"psi must hold {n} elements")
    for t, nm in ((vext, "vext"), (rho, "rho"), (vh, "vh")):
        if t.numel() != int(np.prod(plan.grid)):
            raise ValueError(f"{nm} must hold N1*N2*N3 values")
    o = qm_scf_opts(float(alpha), float(tol), int(max_iter), 0, _opts(**dav_opts))
    eig = np.zeros((plan.nk, nbnd))
    st = qm_scf_stats()
    status = _load().qm_scf_hartree(plan.handle, _dev(vext, torch.float64, "vext"), kw.ctypes.data,
                                    int(nocc), _dev(psi, torch.complex128, "psi"), int(nbnd),
                                    ctypes.byref(o), eig.ctypes.data, _dev(rho, torch.float64, "rho"),
                                    _dev(vh, torch.float64, "vh"), ctypes.byref(st), _stream(stream))
    if status not in (QM_OK, QM_E_NOT_CONVERGED):
        _check(status, plan.handle)
    return eig, st.as_dict(), status


def qm_expm_taylor(plan, k, psi_in, psi_out, nbnd, dt, order, stream=None):
    """psi_out <- sum_{r<=order} (-i dt)^r / r! H^r psi_in (complex128 device tensors)."""
    import torch
    n = plan.band_block_numel(nbnd, k)
    if n is not None and (psi_in.numel() != n or psi_out.numel() != n):
        raise ValueError(f"psi_in/psi_out must hold {n} elements for nbnd={nbnd}, k={k}")
    _check(_load().qm_expm_taylor(plan.handle, int(k), _dev(psi_in, torch.complex128, "psi_in"),
                                  _dev(psi_out, torch.complex128, "psi_out"), int(nbnd), float(dt),
                                  int(order), _stream(stream)), plan.handle)


def qm_td_etrs(plan, vext, kweights, occ, psi, nbnd, dt, order, nsteps, stream=None):
    """nsteps ETRS steps of the Hartree-only model, psi advanced in place."""
    import torch
    kw = np.ascontiguousarray(kweights, np.float64).reshape(-1)
    f = np.ascontiguousarray(occ, np.float64).reshape(-1)
    if kw.size != plan.nk or f.size != plan.nk * nbnd:
        raise ValueError("kweights must hold nk values and occ nk * nbnd")
    if psi.numel() != plan.band_block_numel(nbnd, -1) or vext.numel() != int(np.prod(plan.grid)):
        raise ValueError("psi or vext has the wrong size")
    _check(_load().qm_td_etrs(plan.handle, _dev(vext, torch.float64, "vext"), kw.ctypes.data, f.ctypes.data,
                              _dev(psi, torch.complex128, "psi"), int(nbnd), float(dt), int(order),
                              int(nsteps), _stream(stream)), plan.handle)


def qm_mtxel(plan, kq, psi_kq, nb1, k, psi_k, nb2, miller_g, mtx, stream=None):
    """mtx [nb1, nb2, ng] <- <n k+q| e^{i(q+G).r} |n' k> for the G of miller_g [ng, 3]."""
    import torch
    mg = np.ascontiguousarray(miller_g, np.int32).reshape(-1, 3)
    if psi_kq.numel() != nb1 * int(plan.npw[kq]) or psi_k.numel() != nb2 * int(plan.npw[k]):
        raise ValueError("psi_kq / psi_k sizes do not match nb1, nb2 and the spheres")
    if mtx.numel() != nb1 * nb2 * mg.shape[0]:
        raise ValueError("mtx must hold nb1 * nb2 * ng values")
    _check(_load().qm_mtxel(plan.handle, int(kq), _dev(psi_kq, torch.complex128, "psi_kq"), int(nb1), int(k),
                            _dev(psi_k, torch.complex128, "psi_k"), int(nb2), mg.ctypes.data, int(mg.shape[0]),
                            _dev(mtx, torch.complex128, "mtx"), _stream(stream)), plan.handle)
