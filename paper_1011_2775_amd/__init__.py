"""wcmg: Wilson-clover adaptive-multigrid solver for AMD MI355X (gfx950).

Python face of libwcmg.so.  Every step of the computation runs in the
library's HIP kernels; this module only moves pointers across the C ABI.
Fields are torch tensors on the GPU (complex128, canonical layouts):

  gauge  [Lt][Lz][Ly][Lx][4][3][3]      spinor [nrhs][Lt][Lz][Ly][Lx][4][3]
  coarse [nrhs][Vc][2*Nv]               coarse operator [Vc][9][2Nv][2Nv]
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (F16, F32, F64, OP_DP, OP_FULL, OP_SCHUR, MG_GCR, GCR, BICGSTAB, WcmgError, check)

__all__ = ["Context", "WcmgError", "F64", "F32", "F16", "OP_FULL", "OP_SCHUR", "OP_DP", "MG_GCR", "GCR",
           "BICGSTAB", "default_params"]


def _ptr(t):
    if isinstance(t, torch.Tensor):
        if not t.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(t.data_ptr()), int(t.is_cuda)
    a = np.ascontiguousarray(t)
    return ctypes.c_void_p(a.ctypes.data), 0


def default_params(**kw):
    """Library defaults with keyword overrides; list-valued fields (block, nvec,
    tol, max_iter, restart) per level.  nvec_defl: the number of deflation
    vectors of the coarsest level (coarsest = 2), stored in nvec[nlevels]."""
    p = _lib.MGParams()
    check(_lib.LIB.wcmg_mg_params_default(ctypes.byref(p)))
    defl = kw.pop("nvec_defl", None)
    for k, v in kw.items():
        if k == "block":
            for l, b in enumerate(v):
                for m in range(4):
                    p.block[l][m] = int(b[m])
        elif k in ("nvec", "tol", "max_iter", "restart"):
            arr = getattr(p, k)
            for l, x in enumerate(v):
                arr[l] = x
        else:
            setattr(p, k, v)
    if defl is not None:
        p.nvec[p.nlevels] = int(defl)
    return p


class Context:
    """One library context on the current GPU and torch stream."""

    def __init__(self, lattices, stream=None):
        if isinstance(lattices[0], int):
            lattices = [lattices]
        arr = (_lib.Lattice * len(lattices))()
        self.dims = []
        for k, spec in enumerate(lattices):
            dims, t_bc = (spec, -1) if isinstance(spec[0], int) else (spec[0], spec[1])
            for m in range(4):
                arr[k].dims[m] = int(dims[m])
            arr[k].t_bc = int(t_bc)
            self.dims.append(tuple(int(d) for d in dims))
        if stream is None and torch.cuda.is_available():
            stream = torch.cuda.current_stream().cuda_stream
        h = ctypes.c_void_p()
        check(_lib.LIB.wcmg_create(arr, len(lattices), ctypes.c_void_p(stream or 0), ctypes.byref(h)))
        self.h = h
        self.params = {}

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            _lib.LIB.wcmg_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def volume(self, lat=0):
        return int(np.prod(self.dims[lat]))

    # -- fields ------------------------------------------------------------
    def set_gauge(self, U, lat=0):
        p, dev = _ptr(U)
        check(_lib.LIB.wcmg_set_gauge(self.h, lat, p, dev))

    def set_clover(self, m0, csw, A=None, lat=0):
        if A is None:
            check(_lib.LIB.wcmg_set_clover(self.h, lat, float(m0), float(csw), None, 1))
        else:
            p, dev = _ptr(A)
            check(_lib.LIB.wcmg_set_clover(self.h, lat, float(m0), float(csw), p, dev))

    # -- multigrid -----------------------------------------------------------
    def set_mg_params(self, params, lat=0):
        self.params[lat] = params
        check(_lib.LIB.wcmg_set_mg_params(self.h, lat, ctypes.byref(params)))

    def build_null_vectors(self, level=0, lat=0):
        check(_lib.LIB.wcmg_build_null_vectors(self.h, lat, level))

    def set_null_vectors(self, v, level=0, lat=0):
        p, dev = _ptr(v)
        check(_lib.LIB.wcmg_set_null_vectors(self.h, lat, level, p, int(v.shape[0]), dev))

    def get_null_vectors(self, level=0, lat=0):
        nv = self.params[lat].nvec[level]
        out = torch.empty((nv,) + self._level_shape(level, lat), dtype=torch.complex128, device="cuda")
        check(_lib.LIB.wcmg_get_null_vectors(self.h, lat, level, ctypes.c_void_p(out.data_ptr()), 1))
        return out

    def build_coarse(self, level=0, lat=0):
        check(_lib.LIB.wcmg_build_coarse(self.h, lat, level))

    def coarse_dims(self, level=0, lat=0):
        """Extents of coarse level level+1."""
        d = list(self.dims[lat])
        for l in range(level + 1):
            b = self.params[lat].block[l]
            d = [d[m] // b[m] for m in range(4)]
        return tuple(d)

    def _level_shape(self, level, lat=0):
        """Canonical shape of one vector on level `level` (0: fine spinor, l >= 1: [Vc][2 Nv])."""
        if level == 0:
            return tuple(reversed(self.dims[lat])) + (4, 3)
        return (int(np.prod(self.coarse_dims(level - 1, lat))), 2 * self.params[lat].nvec[level - 1])

    def get_coarse(self, level=0, lat=0):
        n = 2 * self.params[lat].nvec[level]
        Vc = int(np.prod(self.coarse_dims(level, lat)))
        out = np.empty((Vc, 9, n, n), dtype=np.complex128)
        check(_lib.LIB.wcmg_get_coarse(self.h, lat, level, ctypes.c_void_p(out.ctypes.data), 0))
        return out

    # -- operators -------------------------------------------------------------
    def _apply(self, fn, op, prec, inp, lat):
        out = torch.empty_like(inp)
        # lat = -1: all lattices, one right-hand side each, concatenated in lattice order
        nrhs = 1 if lat == -1 else inp.numel() // (self.volume(lat) * 12)
        check(fn(self.h, lat, op, prec, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(inp.data_ptr()), nrhs))
        return out

    def apply_D(self, inp, op=OP_FULL, prec=F64, lat=0):
        return self._apply(_lib.LIB.wcmg_apply_D, op, prec, inp.contiguous(), lat)

    def apply_Ddag(self, inp, op=OP_FULL, prec=F64, lat=0):
        return self._apply(_lib.LIB.wcmg_apply_Ddag, op, prec, inp.contiguous(), lat)

    def restrict(self, fine, level=0, prec=F64, lat=0):
        """Level level -> level+1 restriction R = P^dag gamma5 (prec: arithmetic; complex128 I/O)."""
        shp = self._level_shape(level + 1, lat)
        nrhs = fine.numel() // int(np.prod(self._level_shape(level, lat)))
        out = torch.empty((nrhs,) + shp, dtype=torch.complex128, device=fine.device)
        check(_lib.LIB.wcmg_restrict(self.h, lat, level, prec, ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(fine.contiguous().data_ptr()), nrhs))
        return out

    def prolong(self, coarse, level=0, prec=F64, lat=0):
        nrhs = coarse.shape[0] if coarse.dim() == 3 else 1
        out = torch.empty((nrhs,) + self._level_shape(level, lat), dtype=torch.complex128, device=coarse.device)
        check(_lib.LIB.wcmg_prolong(self.h, lat, level, prec, ctypes.c_void_p(out.data_ptr()),
                                    ctypes.c_void_p(coarse.contiguous().data_ptr()), nrhs))
        return out

    def apply_coarse(self, inp, level=1, op=OP_FULL, prec=F64, lat=0):
        inp = inp.contiguous()
        out = torch.empty_like(inp)
        n = inp.shape[-1]
        Vc = inp.shape[-2]
        nrhs = inp.numel() // (Vc * n)
        check(_lib.LIB.wcmg_apply_coarse(self.h, lat, level, op, prec, ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(inp.data_ptr()), nrhs))
        return out

    def coarse_solve(self, b, level=1, prec=F64, tol=0.1, max_iter=100, restart=30, launch=0, lat=0):
        """Approximate Dhat^-1 b on coarse level `level` (complex128 [Vc][2Nv] device
        vector) by the red-black GCR of the cycle; launch 0: one cooperative launch (the
        one-site kernel where it applies), 1: one launch per kernel, 2: the strided
        cooperative kernel."""
        b = b.contiguous()
        x = torch.empty_like(b)
        st = _lib.Stats()
        check(_lib.LIB.wcmg_coarse_solve(self.h, lat, level, prec, ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(b.data_ptr()), float(tol), int(max_iter), int(restart),
                                         int(launch), ctypes.byref(st)))
        return x, st.as_dict()

    # -- solve -------------------------------------------------------------------
    def solve(self, b, solver=MG_GCR, tol=1e-10, x0=None, lat=0, raise_on_error=True):
        """x with D x = b (canonical complex128 device tensor of nrhs spinors)."""
        return self._solve(_lib.LIB.wcmg_solve, b, solver, tol, x0, lat, raise_on_error)

    def solve_dag(self, b, solver=MG_GCR, tol=1e-10, x0=None, lat=0, raise_on_error=True):
        """x with D^dag x = b, through D^dag = gamma5 D gamma5 (same solver and hierarchy)."""
        return self._solve(_lib.LIB.wcmg_solve_dag, b, solver, tol, x0, lat, raise_on_error)

    def _solve(self, fn, b, solver, tol, x0, lat, raise_on_error):
        b = b.contiguous()
        x = torch.zeros_like(b) if x0 is None else x0.clone().contiguous()
        nrhs = b.numel() // (self.volume(lat) * 12)
        st = (_lib.Stats * nrhs)()
        rc = fn(self.h, lat, solver, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(b.data_ptr()), nrhs, float(tol),
                st)
        if raise_on_error:
            check(rc)
        return x, [s.as_dict() for s in st]

    def force(self, psi, lam, include_clover=True, lat=0):
        """Gauge-link gradient -dRe<lam, D(U) psi>/dU (complex128 [Lt][Lz][Ly][Lx][4][3][3]),
        summed over the right-hand sides of psi and lam."""
        psi = psi.contiguous()
        lam = lam.contiguous()
        if psi.shape != lam.shape or psi.dtype != torch.complex128 or lam.dtype != torch.complex128:
            raise ValueError("psi and lam must be complex128 tensors of the same shape")
        nrhs = psi.numel() // (self.volume(lat) * 12)
        dims = self.dims[lat]
        dU = torch.empty((dims[3], dims[2], dims[1], dims[0], 4, 3, 3), dtype=torch.complex128, device=psi.device)
        check(_lib.LIB.wcmg_force(self.h, lat, ctypes.c_void_p(dU.data_ptr()), ctypes.c_void_p(psi.data_ptr()),
                                  ctypes.c_void_p(lam.data_ptr()), nrhs, int(bool(include_clover))))
        return dU

    # -- global sums -------------------------------------------------------------
    def dot(self, x, y):
        """sum conj(x) y of two device tensors (complex128 or complex64), in FP64."""
        prec = F64 if x.dtype == torch.complex128 else F32
        out = (ctypes.c_double * 2)()
        check(_lib.LIB.wcmg_dot(self.h, prec, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                x.numel(), out))
        return complex(out[0], out[1])

    # -- autotuner -----------------------------------------------------------------
    def autotune(self, on=True):
        check(_lib.LIB.wcmg_autotune(self.h, int(bool(on))))

    def autotune_report(self):
        """The tuned launch shapes: list of dicts (prec, diag, postinv, Vh, nrhs, threads, group, us)."""
        buf = ctypes.create_string_buffer(1 << 16)
        check(_lib.LIB.wcmg_autotune_report(self.h, buf, len(buf)))
        keys = ("prec", "diag", "postinv", "Vh", "nrhs", "threads", "group", "us")
        out = []
        for line in buf.value.decode().splitlines():
            vals = line.split()
            out.append({k: (float(v) if k == "us" else int(v)) for k, v in zip(keys, vals)})
        return out

    # -- timing --------------------------------------------------------------------
    def timer_enable(self, on=True):
        check(_lib.LIB.wcmg_timer_enable(self.h, int(bool(on))))

    def timer_read(self, which=0):
        n = ctypes.c_long()
        ms = ctypes.c_double()
        check(_lib.LIB.wcmg_timer_read(self.h, which, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value
