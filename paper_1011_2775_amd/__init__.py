"""wcmg: Wilson-clover adaptive-multigrid solver for AMD MI355X (gfx950).

Python face of libwcmg.so.  Every step of the computation runs in the
library's HIP kernels; this module only moves pointers across the C ABI.
Fields are torch tensors on the GPU (complex128, canonical layouts):

  gauge  [Lt][Lz][Ly][Lx][4][3][3]      spinor [nrhs][Lt][Lz][Ly][Lx][4][3]
  coarse [nrhs][Vc][2*Nv]               coarse operator [Vc][9][2Nv][2Nv]
"""
import atexit
import ctypes
import sys
import weakref

import numpy as np
import torch

from . import _lib
from ._lib import (F16, F32, F64, OP_DP, OP_FULL, OP_SCHUR, OP_SCHUR_X, MG_GCR, GCR, BICGSTAB, MP_BICGSTAB, CGNR, WcmgError,
                   check)

__all__ = ["Context", "WcmgError", "F64", "F32", "F16", "OP_FULL", "OP_SCHUR", "OP_DP", "OP_SCHUR_X", "MG_GCR", "GCR",
           "BICGSTAB", "MP_BICGSTAB", "CGNR", "default_params"]


def _ptr(t, numel=None, name="buffer"):
    """(pointer, on_device, keep-alive) of a complex128 buffer of `numel`
    elements: a contiguous CUDA or CPU tensor, or anything numpy converts.
    Keep the third value alive until the library call returns."""
    if isinstance(t, torch.Tensor):
        if t.dtype != torch.complex128:
            raise ValueError("%s must be complex128, not %s" % (name, t.dtype))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        if numel is not None and t.numel() != numel:
            raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), numel))
        if t.is_cuda:
            return ctypes.c_void_p(t.data_ptr()), 1, t
        t = t.numpy()
    a = np.ascontiguousarray(t, dtype=np.complex128)
    if numel is not None and a.size != numel:
        raise ValueError("%s has %d elements, expected %d" % (name, a.size, numel))
    return ctypes.c_void_p(a.ctypes.data), 0, a


def _dev(t, unit, name, dtype=torch.complex128):
    """A contiguous CUDA tensor of `dtype` whose element count is a positive
    multiple of `unit`; returns that multiple (the number of right-hand sides)."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must be %s, not %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() == 0 or t.numel() % unit:
        raise ValueError("%s has %d elements, not a positive multiple of %d" % (name, t.numel(), unit))
    return t.numel() // unit


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


# Contexts still open when the interpreter exits are destroyed by an atexit
# handler, while the HIP runtime is certainly alive (atexit handlers run
# before the interpreter tears its modules down, and long before the C
# runtime's exit handlers unload HIP).  During interpreter finalisation
# __del__ makes no library call at all: a context reached only then is left
# to the process exit rather than freed into a runtime that may be gone.
_LIVE = weakref.WeakSet()


@atexit.register
def _close_live_contexts():
    for ctx in list(_LIVE):
        ctx.close()


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
        _LIVE.add(self)

    def close(self):
        """Destroy the library context (synchronises its stream, frees its device memory)."""
        if getattr(self, "h", None) and self.h.value:
            h, self.h = self.h, ctypes.c_void_p()
            check(_lib.LIB.wcmg_destroy(h))
        _LIVE.discard(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        if sys is None or sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def volume(self, lat=0):
        return int(np.prod(self.dims[lat]))

    # -- fields ------------------------------------------------------------
    def set_gauge(self, U, lat=0):
        p, dev, keep = _ptr(U, self.volume(lat) * 36, "gauge field")
        check(_lib.LIB.wcmg_set_gauge(self.h, lat, p, dev))
        del keep

    def set_clover(self, m0, csw, A=None, lat=0):
        if A is None:
            check(_lib.LIB.wcmg_set_clover(self.h, lat, float(m0), float(csw), None, 1))
        else:
            p, dev, keep = _ptr(A, self.volume(lat) * 144, "clover matrix")
            check(_lib.LIB.wcmg_set_clover(self.h, lat, float(m0), float(csw), p, dev))
            del keep

    def set_clover_aniso(self, m0, hop_s, csw_s, csw_t, lat=0):
        """Anisotropic Wilson-clover: spatial hops weighted by hop_s, diagonal m0 + 1 + 3 hop_s,
        clover planes weighted csw_s (spatial) and csw_t (with time)."""
        check(_lib.LIB.wcmg_set_clover_aniso(self.h, lat, float(m0), float(hop_s), float(csw_s), float(csw_t)))

    # -- multigrid -----------------------------------------------------------
    def set_mg_params(self, params, lat=0):
        self.params[lat] = params
        check(_lib.LIB.wcmg_set_mg_params(self.h, lat, ctypes.byref(params)))

    def build_null_vectors(self, level=0, lat=0):
        check(_lib.LIB.wcmg_build_null_vectors(self.h, lat, level))

    def set_null_vectors(self, v, level=0, lat=0):
        nv = int(v.shape[0])
        p, dev, keep = _ptr(v, nv * int(np.prod(self._level_shape(level, lat))), "null vectors")
        check(_lib.LIB.wcmg_set_null_vectors(self.h, lat, level, p, nv, dev))
        del keep

    def get_null_vectors(self, level=0, lat=0):
        nv = self.params[lat].nvec[level]
        out = torch.empty((nv,) + self._level_shape(level, lat), dtype=torch.complex128, device="cuda")
        check(_lib.LIB.wcmg_get_null_vectors(self.h, lat, level, ctypes.c_void_p(out.data_ptr()), 1))
        return out

    def setup_start_vectors(self, seed, nvec, k0=0, level=0, lat=0):
        """The setup's Philox start vectors k0 .. k0+nvec-1 of `level` (canonical, complex128)."""
        out = torch.empty((nvec,) + self._level_shape(level, lat), dtype=torch.complex128, device="cuda")
        check(_lib.LIB.wcmg_setup_start_vectors(self.h, lat, level, int(seed), int(k0), int(nvec),
                                                ctypes.c_void_p(out.data_ptr())))
        return out

    def refine_null_vectors(self, passes=1, iters=4, lat=0):
        """Relax the fine null vectors with the current multigrid cycle and rebuild the hierarchy."""
        check(_lib.LIB.wcmg_refine_null_vectors(self.h, lat, int(passes), int(iters)))

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
        # lat = -1: all lattices, one right-hand side each, concatenated in lattice order
        unit = sum(self.volume(l) for l in range(len(self.dims))) * 12 if lat == -1 else self.volume(lat) * 12
        nrhs = _dev(inp, unit, "input")
        out = torch.empty_like(inp)
        check(fn(self.h, lat, op, prec, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(inp.data_ptr()), nrhs))
        return out

    def apply_D(self, inp, op=OP_FULL, prec=F64, lat=0):
        return self._apply(_lib.LIB.wcmg_apply_D, op, prec, inp.contiguous(), lat)

    def apply_Ddag(self, inp, op=OP_FULL, prec=F64, lat=0):
        return self._apply(_lib.LIB.wcmg_apply_Ddag, op, prec, inp.contiguous(), lat)

    def restrict(self, fine, level=0, prec=F64, lat=0):
        """Level level -> level+1 restriction R = P^dag gamma5 (prec: arithmetic; complex128 I/O)."""
        shp = self._level_shape(level + 1, lat)
        fine = fine.contiguous()
        nrhs = _dev(fine, int(np.prod(self._level_shape(level, lat))), "fine vectors")
        out = torch.empty((nrhs,) + shp, dtype=torch.complex128, device=fine.device)
        check(_lib.LIB.wcmg_restrict(self.h, lat, level, prec, ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(fine.data_ptr()), nrhs))
        return out

    def prolong(self, coarse, level=0, prec=F64, lat=0):
        coarse = coarse.contiguous()
        nrhs = _dev(coarse, int(np.prod(self._level_shape(level + 1, lat))), "coarse vectors")
        out = torch.empty((nrhs,) + self._level_shape(level, lat), dtype=torch.complex128, device=coarse.device)
        check(_lib.LIB.wcmg_prolong(self.h, lat, level, prec, ctypes.c_void_p(out.data_ptr()),
                                    ctypes.c_void_p(coarse.data_ptr()), nrhs))
        return out

    def apply_coarse(self, inp, level=1, op=OP_FULL, prec=F64, lat=0):
        inp = inp.contiguous()
        nrhs = _dev(inp, int(np.prod(self._level_shape(level, lat))), "coarse vectors")
        out = torch.empty_like(inp)
        check(_lib.LIB.wcmg_apply_coarse(self.h, lat, level, op, prec, ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(inp.data_ptr()), nrhs))
        return out

    def coarse_solve(self, b, level=1, prec=F64, tol=0.1, max_iter=100, restart=30, launch=0, lat=0):
        """Approximate Dhat^-1 b on coarse level `level` (complex128 [Vc][2Nv] device
        vector) by the red-black GCR of the cycle; launch 0: one cooperative launch (the
        one-site kernel where it applies), 1: one launch per kernel, 2: the strided
        cooperative kernel."""
        b = b.contiguous()
        if _dev(b, int(np.prod(self._level_shape(level, lat))), "right-hand side") != 1:
            raise ValueError("the coarse solve takes one right-hand side")
        x = torch.empty_like(b)
        st = _lib.Stats()
        check(_lib.LIB.wcmg_coarse_solve(self.h, lat, level, prec, ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(b.data_ptr()), float(tol), int(max_iter), int(restart),
                                         int(launch), ctypes.byref(st)))
        return x, st.as_dict()

    def coarse_solve_noalloc(self, b, level=1, prec=F64, tol=0.1, max_iter=100, restart=30, lat=0):
        """coarse_solve(launch=0) through the allocation-free entry point (every work buffer in
        the library's static device array); x is allocated here, by torch, as the caller."""
        b = b.contiguous()
        if _dev(b, int(np.prod(self._level_shape(level, lat))), "right-hand side") != 1:
            raise ValueError("the coarse solve takes one right-hand side")
        x = torch.empty_like(b)
        st = _lib.Stats()
        check(_lib.LIB.wcmg_coarse_solve_noalloc(self.h, lat, level, prec, ctypes.c_void_p(x.data_ptr()),
                                                 ctypes.c_void_p(b.data_ptr()), float(tol), int(max_iter),
                                                 int(restart), ctypes.byref(st)))
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
        # lat = -1: every lattice, nrhs right-hand sides each, concatenated in lattice order
        nl = len(self.dims) if lat == -1 else 1
        unit = sum(self.volume(l) for l in range(nl)) * 12 if lat == -1 else self.volume(lat) * 12
        nrhs = _dev(b, unit, "right-hand sides")
        x = torch.zeros_like(b) if x0 is None else x0.clone().contiguous()
        if _dev(x, unit, "initial guess") != nrhs:
            raise ValueError("initial guess and right-hand sides differ in size")
        st = (_lib.Stats * (nl * nrhs))()
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
        nrhs = _dev(psi, self.volume(lat) * 12, "psi")
        if psi.shape != lam.shape or _dev(lam, self.volume(lat) * 12, "lam") != nrhs:
            raise ValueError("psi and lam must have the same shape")
        dims = self.dims[lat]
        dU = torch.empty((dims[3], dims[2], dims[1], dims[0], 4, 3, 3), dtype=torch.complex128, device=psi.device)
        check(_lib.LIB.wcmg_force(self.h, lat, ctypes.c_void_p(dU.data_ptr()), ctypes.c_void_p(psi.data_ptr()),
                                  ctypes.c_void_p(lam.data_ptr()), nrhs, int(bool(include_clover))))
        return dU

    # -- global sums -------------------------------------------------------------
    def dot(self, x, y):
        """sum conj(x) y of two device tensors (complex128 or complex64), in FP64."""
        prec = F64 if x.dtype == torch.complex128 else F32
        n = _dev(x, 1, "x", x.dtype if x.dtype in (torch.complex128, torch.complex64) else torch.complex128)
        if _dev(y, 1, "y", x.dtype) != n:
            raise ValueError("x and y differ in length")
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
        """True / 1: time every timed kernel; 2: only the persistent coarse solves; False / 0: off."""
        check(_lib.LIB.wcmg_timer_enable(self.h, 2 if on == 2 and on is not True else int(bool(on))))

    def timer_read(self, which=0):
        n = ctypes.c_long()
        ms = ctypes.c_double()
        check(_lib.LIB.wcmg_timer_read(self.h, which, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value
