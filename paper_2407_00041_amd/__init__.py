"""wdirac: the Wilson-clover Dirac operator of arXiv 2407.00041 (Eq. (1.13)) and
FGMRES (Algorithm 2) on an AMD Instinct MI355X, behind the C ABI of
``include/wdirac.h``.

Python here only marshals arguments: torch supplies device memory and the
current HIP stream; every step runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (ANTIPERIODIC_T, COMPRESS_CLOVER, COMPRESS_LINKS, EVEN_ODD, EUNSUPPORTED, F16S, F32, F64,  # noqa: F401
                   ENONFINITE, ENOTCONV, FGMRES_AMG, FGMRES_F64, FGMRES_SAP,
                   FGMRES_MIXED_F16S, FGMRES_MIXED_F32, WITH_F16, WITH_F32, WdiracError, check)

PRECS = {"f64": F64, "f32": F32, "f16s": F16S}


def _prec(p) -> int:
    return PRECS[p] if isinstance(p, str) else int(p)


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _ptr(t: torch.Tensor) -> int:
    return int(t.data_ptr())


def _host_c128(a, shape_tail):
    if isinstance(a, torch.Tensor):
        a = a.detach().cpu().numpy()
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    assert a.shape[-len(shape_tail):] == tuple(shape_tail), (a.shape, shape_tail)
    return a


class DiracOp:
    """Operator handle: D = A - 1/2 sum hop terms on a periodic 4-D lattice.

    dims = (nT, nZ, nY, nX); links canonical [V, 4, 3, 3] complex128 (host or
    device tensor / ndarray); clover None (build from links when csw != 0) or
    the packed unit-c_sw term [V, 42].  compress_links: two stored rows per
    SU(3) link; compress_clover: each clover chirality block stored as its
    spin-diagonal difference and off-diagonal 3x3 blocks (27 of 36 reals);
    even_odd: also store A(x)^{-1} for the even-odd reduced system.
    """

    def __init__(self, dims, links, m0: float, csw: float = 0.0, clover=None,
                 antiperiodic_t: bool = False, precisions=("f64", "f32", "f16s"),
                 compress_links: bool = False, compress_clover: bool = False, even_odd: bool = False):
        self.lib = _lib.load()
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.m0, self.csw = float(m0), float(csw)
        self.antiperiodic_t = bool(antiperiodic_t)
        flags = ANTIPERIODIC_T if antiperiodic_t else 0
        if compress_links:
            flags |= COMPRESS_LINKS
        self.compress_links = bool(compress_links)
        if compress_clover:
            flags |= COMPRESS_CLOVER
        self.compress_clover = bool(compress_clover)
        if even_odd:
            flags |= EVEN_ODD
        self.even_odd = bool(even_odd)
        if "f32" in precisions:
            flags |= WITH_F32
        if "f16s" in precisions:
            flags |= WITH_F16
        self.precisions = tuple(precisions)
        L = _host_c128(links, (4, 3, 3)).reshape(self.V, 4, 3, 3)
        C = None if clover is None else _host_c128(clover, (42,)).reshape(self.V, 42)
        d = (ctypes.c_int * 4)(*self.dims)
        h = ctypes.c_void_p()
        torch.cuda.init()
        check(self.lib.dirac_create(ctypes.byref(h), d, L.ctypes.data, None if C is None else C.ctypes.data,
                                    self.m0, self.csw, flags), "dirac_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.dirac_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- fields
    def field_bytes(self, prec="f64", nrhs: int = 1) -> int:
        return int(self.lib.dirac_field_bytes(self.handle, _prec(prec), int(nrhs)))

    def empty(self, prec="f64", nrhs: int = 1, device="cuda") -> torch.Tensor:
        """Native field buffer (uint8 tensor of field_bytes)."""
        return torch.empty(self.field_bytes(prec, nrhs), dtype=torch.uint8, device=device)

    def pack(self, canonical: torch.Tensor, prec="f64", out: torch.Tensor | None = None,
             stream=None) -> torch.Tensor:
        """canonical [nrhs, V, 12] (or [V, 12]) complex128 on the device -> native."""
        c = canonical.contiguous()
        assert c.dtype == torch.complex128 and c.is_cuda
        nrhs = c.numel() // (12 * self.V)
        assert nrhs * 12 * self.V == c.numel()
        out = self.empty(prec, nrhs, c.device) if out is None else out
        check(self.lib.dirac_pack(self.handle, _ptr(out), _ptr(c), nrhs, _prec(prec), _stream(stream)),
              "dirac_pack")
        return out

    def unpack(self, native: torch.Tensor, prec="f64", nrhs: int | None = None,
               stream=None) -> torch.Tensor:
        """native -> canonical [nrhs, V, 12] complex128."""
        p = _prec(prec)
        if nrhs is None:
            nrhs = native.numel() * native.element_size() // self.field_bytes(p, 1)
        out = torch.empty((nrhs, self.V, 12), dtype=torch.complex128, device=native.device)
        check(self.lib.dirac_unpack(self.handle, _ptr(out), _ptr(native), nrhs, p, _stream(stream)),
              "dirac_unpack")
        return out

    # ------------------------------------------------------------- even-odd
    def parity_field_bytes(self, prec="f64", nrhs: int = 1) -> int:
        return int(self.lib.dirac_parity_field_bytes(self.handle, _prec(prec), int(nrhs)))

    def empty_parity(self, prec="f64", nrhs: int = 1, device="cuda") -> torch.Tensor:
        """Native parity-field buffer (V/2 sites) of parity_field_bytes."""
        return torch.empty(self.parity_field_bytes(prec, nrhs), dtype=torch.uint8, device=device)

    def split(self, full: torch.Tensor, prec="f64", nrhs: int = 1, stream=None):
        """Native full field -> (even, odd) native parity fields."""
        e, o = self.empty_parity(prec, nrhs, full.device), self.empty_parity(prec, nrhs, full.device)
        check(self.lib.dirac_parity_split(self.handle, _ptr(e), _ptr(o), _ptr(full), int(nrhs), _prec(prec),
                                          _stream(stream)), "dirac_parity_split")
        return e, o

    def merge(self, even: torch.Tensor, odd: torch.Tensor, prec="f64", nrhs: int = 1, stream=None):
        """(even, odd) native parity fields -> native full field."""
        f = self.empty(prec, nrhs, even.device)
        check(self.lib.dirac_parity_merge(self.handle, _ptr(f), _ptr(even), _ptr(odd), int(nrhs), _prec(prec),
                                          _stream(stream)), "dirac_parity_merge")
        return f

    def apply_schur_native(self, out, inp, tmp, nrhs: int = 1, prec="f64", dagger: bool = False, stream=None):
        """out = S inp (S^H with dagger), S = A_ee - H_eo A_oo^-1 H_oe; tmp: nrhs odd fields."""
        check(self.lib.dirac_apply_schur(self.handle, _ptr(out), _ptr(inp), _ptr(tmp), int(nrhs), _prec(prec),
                                         int(bool(dagger)), _stream(stream)), "dirac_apply_schur")
        return out

    def schur_prepare_native(self, bhat, b_even, b_odd, tmp, nrhs: int = 1, prec="f64", stream=None):
        """bhat = b_e - H_eo A_oo^-1 b_o."""
        check(self.lib.dirac_schur_prepare(self.handle, _ptr(bhat), _ptr(b_even), _ptr(b_odd), _ptr(tmp),
                                           int(nrhs), _prec(prec), _stream(stream)), "dirac_schur_prepare")
        return bhat

    def schur_reconstruct_native(self, x_odd, x_even, b_odd, nrhs: int = 1, prec="f64", stream=None):
        """x_o = A_oo^-1 (b_o - H_oe x_e)."""
        check(self.lib.dirac_schur_reconstruct(self.handle, _ptr(x_odd), _ptr(x_even), _ptr(b_odd), int(nrhs),
                                               _prec(prec), _stream(stream)), "dirac_schur_reconstruct")
        return x_odd

    # ---------------------------------------------------------------- applies
    def apply_native(self, out: torch.Tensor, inp: torch.Tensor, nrhs: int = 1, prec="f64",
                     dagger: bool = False, stream=None) -> torch.Tensor:
        f = self.lib.dirac_apply_adjoint if dagger else self.lib.dirac_apply
        check(f(self.handle, _ptr(out), _ptr(inp), int(nrhs), _prec(prec), _stream(stream)),
              "dirac_apply_adjoint" if dagger else "dirac_apply")
        return out

    def apply_batched(self, batches, prec="f32", dagger: bool = False, stream=None):
        """batches: list of (out, inp, nrhs) native buffers; one launch."""
        arr = (_lib.DiracBatch * len(batches))()
        for k, (o, i, n) in enumerate(batches):
            arr[k].out, arr[k].inp, arr[k].nrhs = _ptr(o), _ptr(i), int(n)
        check(self.lib.dirac_apply_batched(self.handle, arr, len(batches), _prec(prec), int(bool(dagger)),
                                           _stream(stream)), "dirac_apply_batched")

    def apply(self, psi: torch.Tensor, prec="f64", dagger: bool = False) -> torch.Tensor:
        """Canonical in, canonical out (pack -> apply -> unpack), for convenience."""
        shape = psi.shape
        c = psi.reshape(-1, self.V, 12)
        nrhs = c.shape[0]
        a = self.pack(c, prec)
        b = self.empty(prec, nrhs, c.device)
        self.apply_native(b, a, nrhs, prec, dagger)
        return self.unpack(b, prec, nrhs).reshape(shape)

    @staticmethod
    def sap_params(block=(4, 4, 4, 4), cycles: int = 1, mr_iters: int = 4, additive: bool = False, prec="f32"):
        """SAP parameters (see dirac_sap): block extents (T, Z, Y, X), Schwarz cycles,
        minimal-residual steps per block solve, additive or red-black, block precision."""
        return _lib.SapParams((ctypes.c_int * 4)(*[int(b) for b in block]), int(cycles), int(mr_iters),
                              int(bool(additive)), _prec(prec))

    @classmethod
    def _params(cls, restart, tol, maxit, mode, inner_restart, inner_tol, inner_maxit, graph=False, wave=0,
                schur=False, sap=None, amg=None):
        modes = {"f64": FGMRES_F64, "mixed_f32": FGMRES_MIXED_F32, "mixed_f16s": FGMRES_MIXED_F16S,
                 "sap": FGMRES_SAP, "amg": FGMRES_AMG}
        sp = cls.sap_params(**(sap or {}))
        return _lib.FgmresParams(int(restart), float(tol), int(maxit),
                                 modes[mode] if isinstance(mode, str) else int(mode),
                                 int(inner_restart), float(inner_tol), int(inner_maxit), int(bool(graph)), int(wave),
                                 int(bool(schur)), sp, amg.handle if amg is not None else None)

    def workspace_bytes(self, nrhs: int = 1, restart: int = 20, mode="f64", inner_restart: int = 30,
                        wave: int = 0, schur: bool = False, sap=None, amg=None) -> int:
        p = self._params(restart, 1e-10, 1, mode, inner_restart, 1e-2, 1, wave=wave, schur=schur, sap=sap, amg=amg)
        n = int(self.lib.fgmres_workspace_bytes(self.handle, ctypes.byref(p), int(nrhs)))
        if n == 0:
            raise WdiracError(-1, "fgmres_workspace_bytes")
        return n

    def solve(self, b: torch.Tensor, nrhs: int = 1, x0: torch.Tensor | None = None, restart: int = 20,
              tol: float = 1e-10, maxit: int = 10000, mode="f64", inner_restart: int = 30,
              inner_tol: float = 1e-2, inner_maxit: int = 30, work: torch.Tensor | None = None, stream=None,
              graph: bool = False, wave: int = 0, schur: bool = False, sap=None, amg=None):
        """FGMRES for D x = b (b native FP64, nrhs fields).  mode: "f64", "mixed_f32",
        "mixed_f16s", or "sap" (M_j^{-1} = SAP with the keyword arguments of
        sap_params in ``sap``).  ``work`` may be a reusable device buffer of at
        least workspace_bytes(...) bytes.  ``graph``: run the inner cycles of the
        mixed modes as captured HIP graphs.  ``wave``: solve the right-hand sides
        in consecutive groups of this size (workspace for one group); 0 lets the
        library size the groups from the free device memory, or from ``work``
        when it is given.
        ``schur``: solve the even-odd reduced system (operator built with
        even_odd=True) and reconstruct the odd sites; tol stays relative to the
        full system's initial residual.
        ``amg``: a TwoLevel of this operator, the preconditioner of mode "amg".
        Returns (x native FP64, per-RHS stats dicts, status); status is
        ENONFINITE when a right-hand side met NaN/Inf (its stats say
        ``nonfinite``), ENOTCONV when one reached maxit."""
        p = self._params(restart, tol, maxit, mode, inner_restart, inner_tol, inner_maxit, graph, wave, schur, sap,
                         amg)
        nbytes = int(self.lib.fgmres_workspace_bytes(self.handle, ctypes.byref(p), int(nrhs)))
        if nbytes == 0:
            raise WdiracError(-1, "fgmres_workspace_bytes")
        if work is None:
            work = torch.empty(nbytes, dtype=torch.uint8, device=b.device)
        elif wave > 0 and work.numel() * work.element_size() < nbytes:
            raise ValueError(f"workspace of {work.numel()} bytes is smaller than {nbytes}")
        else:
            # wave = 0 with a given workspace: the library fits as many right-hand sides per wave as it holds
            nbytes = work.numel() * work.element_size()
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        stats = (_lib.FgmresStats * int(nrhs))()
        rc = check(self.lib.fgmres_solve(self.handle, _ptr(x), _ptr(b), int(nrhs), ctypes.byref(p), stats,
                                         _ptr(work), nbytes, _stream(stream)), "fgmres_solve")
        out = []
        for s in stats:
            out.append({"applies": s.applies, "inner_applies": s.inner_applies, "restarts": s.restarts,
                        "converged": bool(s.converged), "breakdown": bool(s.breakdown),
                        "nonfinite": bool(s.nonfinite), "wave": s.wave,
                        "true_residual": s.true_residual, "seconds": s.seconds,
                        "seconds_apply": s.seconds_apply, "seconds_precond": s.seconds_precond,
                        "seconds_ortho": s.seconds_ortho,
                        "hist": [s.hist[i] for i in range(s.nhist)]})
        return x, out, rc

    def sap(self, b: torch.Tensor, nrhs: int = 1, x: torch.Tensor | None = None, stream=None, **kw) -> torch.Tensor:
        """x = SAP(b) from x = 0 (dirac_sap); b native FP64 with nrhs fields; kw: sap_params."""
        p = self.sap_params(**kw)
        nb = int(self.lib.dirac_sap_workspace_bytes(self.handle, ctypes.byref(p), int(nrhs)))
        work = torch.empty(max(nb, 16), dtype=torch.uint8, device=b.device)
        x = torch.empty_like(b) if x is None else x
        check(self.lib.dirac_sap(self.handle, _ptr(x), _ptr(b), int(nrhs), ctypes.byref(p), _ptr(work), nb,
                                 _stream(stream)), "dirac_sap")
        return x

    def autotune(self, prec="f64", nrhs: int = 1, stream=None) -> dict:
        """Time candidate launch configurations and keep the fastest (dirac_autotune)."""
        cfg = (ctypes.c_int * 5)()
        us = ctypes.c_double()
        check(self.lib.dirac_autotune(self.handle, _prec(prec), int(nrhs), cfg, ctypes.byref(us), _stream(stream)),
              "dirac_autotune")
        return {"order": cfg[0], "block": cfg[1], "tchunk": cfg[2], "nr": cfg[3], "persistent": cfg[4],
                "us": us.value}

    def force(self, eta: torch.Tensor, x: torch.Tensor, nrhs: int = 1, raw: bool = False,
              stream=None) -> torch.Tensor:
        """dL/dU for L = Re sum <eta, D x>; eta, x native FP64.  [V, 4, 3, 3] c128."""
        out = torch.empty((self.V, 4, 3, 3), dtype=torch.complex128, device=x.device)
        nb = int(self.lib.dirac_force_workspace_bytes(self.handle))
        work = torch.empty(max(nb, 1), dtype=torch.uint8, device=x.device)
        check(self.lib.dirac_force(self.handle, _ptr(out), _ptr(eta), _ptr(x), int(nrhs), int(bool(raw)),
                                   _ptr(work), nb, _stream(stream)), "dirac_force")
        return out


class TwoLevel:
    """The two-level multigrid of an operator (dirac_amg_*): setup at
    construction from the caller's initial test vectors (device, native FP64,
    ntv fields), then restriction, prolongation, the coarse operator, the
    coarse solve and the preconditioner M.  ``smoother`` holds sap_params
    keywords; ``prec`` is the storage of P ("f64" or "f32")."""

    def __init__(self, op: DiracOp, testvecs: torch.Tensor, agg=(4, 4, 4, 4), ntv: int = 8, init_iters: int = 3,
                 setup_iters: int = 1, smoother=None, coarse_restart: int = 30, coarse_maxit: int = 1000,
                 coarse_tol: float = 0.05, prec="f64", stream=None):
        self.lib = _lib.load()
        self.op = op
        self.N = int(ntv)
        sp = DiracOp.sap_params(**(smoother or {}))
        self.params = _lib.AmgParams((ctypes.c_int * 4)(*[int(a) for a in agg]), self.N, int(init_iters),
                                     int(setup_iters), sp, int(coarse_restart), int(coarse_maxit), float(coarse_tol),
                                     _prec(prec))
        h = ctypes.c_void_p()
        check(self.lib.dirac_amg_create(ctypes.byref(h), op.handle, ctypes.byref(self.params), _ptr(testvecs),
                                        _stream(stream)), "dirac_amg_create")
        self.handle = h
        cd = (ctypes.c_int * 4)()
        nu = ctypes.c_int()
        check(self.lib.dirac_amg_sizes(self.handle, cd, ctypes.byref(nu), None), "dirac_amg_sizes")
        self.coarse_dims = tuple(int(c) for c in cd)
        self.Vc = int(np.prod(self.coarse_dims))
        self.unknowns = int(nu.value)

    def close(self):
        if getattr(self, "handle", None):
            self.lib.dirac_amg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self) -> dict:
        st = (ctypes.c_longlong * 2)()
        check(self.lib.dirac_amg_sizes(self.handle, None, None, st), "dirac_amg_sizes")
        return {"coarse_solves": int(st[0]), "coarse_applies": int(st[1])}

    def empty_coarse(self, nrhs: int = 1, device="cuda") -> torch.Tensor:
        """Coarse vectors [nrhs, Vc, 2, N] complex128."""
        return torch.empty((int(nrhs), self.Vc, 2, self.N), dtype=torch.complex128, device=device)

    def restrict(self, fine: torch.Tensor, nrhs: int = 1, stream=None) -> torch.Tensor:
        out = self.empty_coarse(nrhs, fine.device)
        check(self.lib.dirac_amg_restrict(self.handle, _ptr(out), _ptr(fine), int(nrhs), _stream(stream)),
              "dirac_amg_restrict")
        return out

    def prolong(self, coarse: torch.Tensor, nrhs: int = 1, stream=None) -> torch.Tensor:
        out = self.op.empty("f64", nrhs, coarse.device)
        check(self.lib.dirac_amg_prolong(self.handle, _ptr(out), _ptr(coarse.contiguous()), int(nrhs),
                                         _stream(stream)), "dirac_amg_prolong")
        return out

    def coarse_apply(self, coarse: torch.Tensor, nrhs: int = 1, stream=None) -> torch.Tensor:
        x = coarse.contiguous()
        out = torch.empty_like(x)
        check(self.lib.dirac_amg_coarse_apply(self.handle, _ptr(out), _ptr(x), int(nrhs), _stream(stream)),
              "dirac_amg_coarse_apply")
        return out

    def coarse_solve(self, b: torch.Tensor, stream=None):
        bb = b.contiguous()
        x = torch.empty_like(bb)
        it = ctypes.c_longlong()
        check(self.lib.dirac_amg_coarse_solve(self.handle, _ptr(x), _ptr(bb), ctypes.byref(it), _stream(stream)),
              "dirac_amg_coarse_solve")
        return x, int(it.value)

    def precond(self, r: torch.Tensor, nrhs: int = 1, stream=None) -> torch.Tensor:
        z = torch.empty_like(r)
        check(self.lib.dirac_amg_precond(self.handle, _ptr(z), _ptr(r), int(nrhs), _stream(stream)),
              "dirac_amg_precond")
        return z

    def export(self, what: str, stream=None) -> torch.Tensor:
        """"test_vectors" / "interpolation" (ntv native FP64 fields) or "coarse_operator"
        ([Vc, 5, 2N, 2N] complex128)."""
        dev = torch.device("cuda", torch.cuda.current_device())
        if what == "coarse_operator":
            out = torch.empty((self.Vc, 5, 2 * self.N, 2 * self.N), dtype=torch.complex128, device=dev)
            code = _lib.AMG_COARSE_OPERATOR
        else:
            out = self.op.empty("f64", self.N, dev)
            code = _lib.AMG_TEST_VECTORS if what == "test_vectors" else _lib.AMG_INTERPOLATION
        check(self.lib.dirac_amg_export(self.handle, code, _ptr(out), _stream(stream)), "dirac_amg_export")
        return out


def tune_set(key: str, value: int) -> None:
    """Set a process-wide launch parameter of the stencil (see dirac_tune_set)."""
    check(_lib.load().dirac_tune_set(key.encode(), int(value)), "dirac_tune_set")


def tune_get(key: str) -> int:
    v = ctypes.c_int()
    check(_lib.load().dirac_tune_get(key.encode(), ctypes.byref(v)), "dirac_tune_get")
    return int(v.value)


TUNE_KEYS = ("block", "order", "tchunk", "persistent_blocks", "nr_f64", "nr_f32", "nr_f16s", "explicit")


def clover_term(dims, links_dev: torch.Tensor, stream=None) -> torch.Tensor:
    """Unit-c_sw clover term [V, 42] c128 built on the device from device links."""
    lib = _lib.load()
    L = links_dev.contiguous()
    assert L.dtype == torch.complex128 and L.is_cuda
    V = int(np.prod(dims))
    out = torch.empty((V, 42), dtype=torch.complex128, device=L.device)
    d = (ctypes.c_int * 4)(*[int(x) for x in dims])
    check(lib.dirac_clover_term(d, _ptr(L), _ptr(out), _stream(stream)), "dirac_clover_term")
    return out
