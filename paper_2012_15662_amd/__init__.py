"""RI-PNOF7 hot path on MI355X: Python binding of librif.so.

Argument marshalling only: every step of the computation runs in the HIP
kernels of librif.so.  PyTorch provides device memory and the stream; there
is no CPU fallback -- if the library is missing or a tensor is not on the GPU
the call raises.

    import paper_2012_15662_amd as rif
    ctx = rif.Context()                       # launches on torch's current stream
    out = ctx.build(b, C, H, occ, pair_of, n_pairs, n_cwo)   # all steps once
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref

__all__ = [
    "Context", "Batch", "Instance", "OnProblem", "OnSet", "OptParams", "OptResult", "RifError", "load_library", "LIB_PATH", "FP64", "FP32", "BF16X3", "BF16X6",
    "FP16X3", "PNOF7", "PNOF5", "EIG_AUTO", "EIG_SYEVD", "EIG_TRD", "EIG_DC", "EXPORTS",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librif.so")

FP64, FP32, BF16X3, BF16X6, FP16X3 = 0, 1, 2, 3, 4
PNOF7, PNOF5 = 0, 1
EIG_AUTO, EIG_SYEVD, EIG_TRD, EIG_DC = 0, 1, 2, 3
_STATUS = {0: "RIF_OK", -1: "RIF_EINVAL", -2: "RIF_ENOMEM", -3: "RIF_EHIP", -4: "RIF_ENOTSUP"}

_vp, _i, _d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
class Instance(ctypes.Structure):
    """struct rif_instance (include/rif.h)."""
    _fields_ = [(n, ctypes.c_int) for n in ("n_bf", "n_aux", "n_pairs", "n_cwo", "n_mo")] + \
               [(n, ctypes.c_void_p) for n in ("b", "C", "H", "occ", "pair_of", "b_half", "b_mo", "d", "J",
                                               "K", "Jn", "Kn", "energy", "lambda_", "grad", "b_split")]


class OnProblem(ctypes.Structure):
    """struct rif_on_problem (include/rif.h)."""
    _fields_ = [(n, ctypes.c_int) for n in ("n_pairs", "n_cwo", "n_omega", "functional", "max_it", "row0")] + \
               [("tol", ctypes.c_double)] + \
               [(n, ctypes.c_void_p) for n in ("Hpp", "J", "K", "pair_of", "gamma", "occ", "energy", "iters",
                                               "status", "work")]


class OptParams(ctypes.Structure):
    """struct rif_opt_params (include/rif.h)."""
    _fields_ = [(n, ctypes.c_int) for n in ("max_outer", "max_inner", "on_max_it", "init_gamma")] + \
               [(n, ctypes.c_double) for n in ("tol_grad", "tol_energy", "on_tol")]


class OptResult(ctypes.Structure):
    """struct rif_opt_result (include/rif.h)."""
    _fields_ = [(n, ctypes.c_int) for n in ("outer", "inner_total", "on_iters_total", "on_status", "status")] + \
               [(n, ctypes.c_double) for n in ("energy", "max_grad", "ms_on", "ms_build", "ms_orbital")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


# name -> (restype, argtypes); mirrors include/rif.h
EXPORTS = {
    "rif_create": (_i, [ctypes.POINTER(_vp), _i, _vp]),
    "rif_destroy": (None, [_vp]),
    "rif_last_error": (ctypes.c_char_p, [_vp]),
    "rif_set_stream": (_i, [_vp, _vp]),
    "rif_sync": (_i, [_vp]),
    "rif_set_workspace_limit": (_i, [_vp, ctypes.c_ulonglong]),
    "rif_transform": (_i, [_vp, _i, _i, _i, _i, _vp, _vp, _i, _vp, _vp, _vp]),
    "rif_jk_mo": (_i, [_vp, _i, _i, _vp, _vp, _i, _vp, _vp]),
    "rif_jk_mo_noalloc": (_i, [_vp, _i, _i, _vp, _vp, _i, _vp, _vp]),
    "rif_jk_ao_per_mo": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp, _i, _vp, _vp]),
    "pnof7_energy_grad": (_i, [_vp, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i,
                               _vp, _vp, _vp]),
    "pnof_energy_grad": (_i, [_vp, _i, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                              _i, _vp, _vp, _vp]),
    "rif_build": (_i, [_vp, ctypes.POINTER(Instance), _i, _i]),
    "rif_build_direct": (_i, [_vp, ctypes.POINTER(Instance), _i, _i]),
    "rif_eri4_bytes": (ctypes.c_ulonglong, [_i]),
    "rif_eri4_from_b": (_i, [_vp, _i, _i, _vp, _vp]),
    "rif_jk_4c": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp]),
    "rif_presplit_b_bytes": (ctypes.c_ulonglong, [_i, _i, _i]),
    "rif_presplit_b": (_i, [_vp, _i, _i, _vp, _i, _vp]),
    "rif_batch_create": (_i, [_vp, _i, ctypes.POINTER(Instance), _i, _i, ctypes.POINTER(_vp)]),
    "rif_batch_run": (_i, [_vp, _i]),
    "rif_batch_destroy": (None, [_vp]),
    "rif_on_work_size": (ctypes.c_long, [_i, _i, _i]),
    "rif_hpp": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp]),
    "rif_on_optimize": (_i, [_vp, _i, ctypes.POINTER(OnProblem)]),
    "rif_on_features": (_i, [_vp, _i, ctypes.POINTER(OnProblem), _vp, _vp, _vp, _vp, _vp]),
    "rif_on_warmstart": (_i, [_vp, _i, ctypes.POINTER(OnProblem), _vp]),
    "rif_mlp_n_params": (ctypes.c_long, []),
    "rif_mlp_forward": (_i, [_vp, _i, _vp, _vp, _vp, _vp, _vp, _vp]),
    "rif_mlp_backward": (_i, [_vp, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "rif_adam": (_i, [_vp, _i, _vp, _vp, _vp, _vp, _i, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                      ctypes.c_float]),
    "rif_prepare_b": (_i, [_vp, _i, _i, _vp, _vp, _d, _vp, _vp, _vp, _vp, _vp]),
    "rif_orbital_step": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp, _vp, _vp]),
    "rif_set_eigensolver": (_i, [_vp, _i, _i]),
    "rif_set_wait_limit": (_i, [_vp, ctypes.c_longlong]),
    "rif_pnof_optimize": (_i, [_vp, ctypes.POINTER(Instance), _i, _i, ctypes.POINTER(OptParams), _vp, _vp, _vp,
                               ctypes.POINTER(OptResult), _vp, _vp, _i]),
    "rif_autotune": (_i, [_vp, _i]),
    "rif_set_tile_variant": (_i, [_vp, _i]),
    "rif_tune_report": (_i, [_vp, ctypes.c_char_p, _i]),
    "rif_tune_load": (_i, [_vp, ctypes.c_char_p]),
    "rif_profile_enable": (_i, [_vp, _i]),
    "rif_profile_report": (_i, [_vp, ctypes.c_char_p, _i]),
    "rif_profile_only": (_i, [_vp, ctypes.c_char_p]),
}

_lib = None

# Live contexts and batches, released by an exit hook while the HIP runtime is
# still up: a finaliser that runs during interpreter teardown could otherwise
# call into the runtime after its own exit handlers.
_live_batches: "weakref.WeakSet" = weakref.WeakSet()
_live_contexts: "weakref.WeakSet" = weakref.WeakSet()


@atexit.register
def _release_all():
    for b in list(_live_batches):
        b.close()
    for c in list(_live_contexts):
        c.close()




class RifError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


def load_library(path: str = LIB_PATH):
    """Load librif.so and declare its signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run paper_2012_15662_amd/build.py "
                          "(or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path == LIB_PATH:
        _lib = lib
    return lib


def _ptr(t, name, dtype=None, numel=None):
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor on the GPU")
    if not t.is_cuda:
        raise ValueError(f"{name}: tensor must be on the GPU (no CPU path exists)")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous (row-major)")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name}: needs at least {numel} elements, has {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One rif_ctx.  `stream`: a torch.cuda.Stream, a raw hipStream_t int, or
    None for torch's current stream on `device`."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = load_library()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        raw = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        h = ctypes.c_void_p()
        st = self.lib.rif_create(ctypes.byref(h), device, ctypes.c_void_p(raw))
        if st != 0:
            raise RifError(st, "rif_create failed")
        self.h = h
        _live_contexts.add(self)

    def close(self):
        if getattr(self, "h", None):
            for b in list(_live_batches):   # a batch holds this context's stream
                if b.ctx is self:
                    b.close()
            self.lib.rif_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # the default argument keeps the check reachable after module teardown
        if _finalizing():
            return   # the exit hook has released every context still open
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        if st != 0:
            raise RifError(st, self.lib.rif_last_error(self.h).decode())

    # ---- plain ABI calls -------------------------------------------------
    def sync(self):
        self._chk(self.lib.rif_sync(self.h))

    def set_workspace_limit(self, nbytes: int):
        self._chk(self.lib.rif_set_workspace_limit(self.h, nbytes))

    def transform(self, b, C, n_omega, prec=FP64, b_half=None, b_mo=None, d=None):
        import torch
        n_aux, n_bf, _ = b.shape
        n_mo = C.shape[1]
        dt = torch.float64 if prec == FP64 else torch.float32
        dev = b.device
        if b_half is None:
            b_half = torch.empty((n_omega, n_aux, n_bf), dtype=dt, device=dev)
        if b_mo is None:
            b_mo = torch.empty((n_aux, n_omega, n_omega), dtype=dt, device=dev)
        if d is None:
            d = torch.empty((n_aux, n_omega), dtype=torch.float64, device=dev)
        self._chk(self.lib.rif_transform(
            self.h, n_bf, n_aux, n_omega, n_mo, _ptr(b, "b", torch.float64, n_aux * n_bf * n_bf),
            _ptr(C, "C", torch.float64, n_bf * n_mo), prec,
            _ptr(b_half, "b_half", dt, n_omega * n_aux * n_bf),
            _ptr(b_mo, "b_mo", dt, n_aux * n_omega * n_omega),
            _ptr(d, "d", torch.float64, n_aux * n_omega)))
        return b_half, b_mo, d

    def jk_mo(self, b_mo, d, prec=FP64, J=None, K=None):
        import torch
        n_aux, n_omega, _ = b_mo.shape
        dt = torch.float64 if prec == FP64 else torch.float32
        if J is None:
            J = torch.empty((n_omega, n_omega), dtype=torch.float64, device=d.device)
        if K is None:
            K = torch.empty((n_omega, n_omega), dtype=torch.float64, device=d.device)
        self._chk(self.lib.rif_jk_mo(
            self.h, n_aux, n_omega, _ptr(b_mo, "b_mo", dt, n_aux * n_omega * n_omega),
            _ptr(d, "d", torch.float64, n_aux * n_omega), prec,
            _ptr(J, "J", torch.float64, n_omega * n_omega),
            _ptr(K, "K", torch.float64, n_omega * n_omega)))
        return J, K

    def jk_mo_noalloc(self, b_mo, d, J, K, prec=FP64):
        """rif_jk_mo_noalloc: J and K into the caller's buffers with the
        library's static scratch (nothing is allocated)."""
        import torch
        n_aux, n_omega, _ = b_mo.shape
        dt = torch.float64 if prec == FP64 else torch.float32
        self._chk(self.lib.rif_jk_mo_noalloc(
            self.h, n_aux, n_omega, _ptr(b_mo, "b_mo", dt, n_aux * n_omega * n_omega),
            _ptr(d, "d", torch.float64, n_aux * n_omega), prec,
            _ptr(J, "J", torch.float64, n_omega * n_omega),
            _ptr(K, "K", torch.float64, n_omega * n_omega)))
        return J, K

    def jk_ao_per_mo(self, b, b_half, d, prec=FP64, Jn=None, Kn=None):
        import torch
        n_aux, n_bf, _ = b.shape
        n_omega = b_half.shape[0]
        dt = torch.float64 if prec == FP64 else torch.float32
        if Jn is None:
            Jn = torch.empty((n_omega, n_bf, n_bf), dtype=dt, device=b.device)
        if Kn is None:
            Kn = torch.empty((n_omega, n_bf, n_bf), dtype=dt, device=b.device)
        self._chk(self.lib.rif_jk_ao_per_mo(
            self.h, n_bf, n_aux, n_omega, _ptr(b, "b", torch.float64, n_aux * n_bf * n_bf),
            _ptr(b_half, "b_half", dt, n_omega * n_aux * n_bf),
            _ptr(d, "d", torch.float64, n_aux * n_omega), prec,
            _ptr(Jn, "Jn", dt, n_omega * n_bf * n_bf), _ptr(Kn, "Kn", dt, n_omega * n_bf * n_bf)))
        return Jn, Kn

    def energy_grad(self, H, C, occ, pair_of, n_pairs, n_cwo, J, K, Jn, Kn, prec=FP64,
                    functional=PNOF7, energy=None, lam=None, grad=None):
        import torch
        n_bf, n_mo = C.shape
        n_omega = n_pairs * (1 + n_cwo)
        dev = C.device
        dt = torch.float64 if prec == FP64 else torch.float32
        if energy is None:
            energy = torch.empty((1,), dtype=torch.float64, device=dev)
        if lam is None:
            lam = torch.empty((n_mo, n_omega), dtype=torch.float64, device=dev)
        if grad is None:
            grad = torch.empty((n_mo, n_mo), dtype=torch.float64, device=dev)
        self._chk(self.lib.pnof_energy_grad(
            self.h, functional, n_bf, n_mo, n_pairs, n_cwo,
            _ptr(pair_of, "pair_of", torch.int32, n_omega), _ptr(H, "H", torch.float64, n_bf * n_bf),
            _ptr(C, "C", torch.float64, n_bf * n_mo), _ptr(occ, "occ", torch.float64, n_omega),
            _ptr(J, "J", torch.float64, n_omega * n_omega), _ptr(K, "K", torch.float64, n_omega * n_omega),
            _ptr(Jn, "Jn", dt, n_omega * n_bf * n_bf), _ptr(Kn, "Kn", dt, n_omega * n_bf * n_bf), prec,
            _ptr(energy, "energy", torch.float64, 1), _ptr(lam, "lambda", torch.float64, n_mo * n_omega),
            _ptr(grad, "grad", torch.float64, n_mo * n_mo)))
        return energy, lam, grad

    # ---- the conventional four-centre path (Table 1) -----------------------
    def eri4_from_b(self, b, eri=None):
        """rif_eri4_from_b: (mu nu|sigma lambda) = sum_l b b with the first pair
        packed, as a flat FP64 tensor of rif_eri4_bytes(n_bf) / 8 elements."""
        import torch
        n_aux, n_bf, _ = b.shape
        n = int(self.lib.rif_eri4_bytes(n_bf)) // 8
        if n == 0:
            raise RifError(-1, "rif_eri4_bytes: bad n_bf")
        if eri is None:
            eri = torch.empty(n, dtype=torch.float64, device=b.device)
        self._chk(self.lib.rif_eri4_from_b(self.h, n_bf, n_aux, _ptr(b, "b", torch.float64, n_aux * n_bf * n_bf),
                                           _ptr(eri, "eri", torch.float64, n)))
        return eri

    def jk_4c(self, eri, C, n_omega, out=None):
        """rif_jk_4c: Table 1 steps 1-3 from the packed integrals; returns a
        dict with Jn, Kn [n_omega][n_bf][n_bf] and J, K [n_omega][n_omega]."""
        import torch
        n_bf, n_mo = C.shape
        f64 = torch.float64
        o = out if out is not None else {}
        for k, shp in (("Jn", (n_omega, n_bf, n_bf)), ("Kn", (n_omega, n_bf, n_bf)), ("J", (n_omega, n_omega)),
                       ("K", (n_omega, n_omega))):
            if o.get(k) is None:
                o[k] = torch.empty(shp, dtype=f64, device=C.device)
        n = int(self.lib.rif_eri4_bytes(n_bf)) // 8
        self._chk(self.lib.rif_jk_4c(
            self.h, n_bf, n_omega, n_mo, _ptr(eri, "eri", f64, n), _ptr(C, "C", f64, n_bf * n_mo),
            _ptr(o["Jn"], "Jn", f64, n_omega * n_bf * n_bf), _ptr(o["Kn"], "Kn", f64, n_omega * n_bf * n_bf),
            _ptr(o["J"], "J", f64, n_omega * n_omega), _ptr(o["K"], "K", f64, n_omega * n_omega)))
        return o

    # ---- one build: every hot-path step once -----------------------------
    def presplit_b(self, b, prec, out=None):
        """rif_presplit_b: b stored once for a reduced-precision mode (a byte
        tensor of rif_presplit_b_bytes), to pass as b_split to build calls in
        that mode."""
        import torch
        n_aux, n_bf, _ = b.shape
        nbytes = int(self.lib.rif_presplit_b_bytes(n_bf, n_aux, prec))
        if nbytes == 0:
            raise RifError(-4, "rif_presplit_b: FP32, BF16x3, BF16x6 or FP16x3 only")
        if out is None:
            out = torch.empty(nbytes, dtype=torch.uint8, device=b.device)
        self._chk(self.lib.rif_presplit_b(self.h, n_bf, n_aux, _ptr(b, "b", torch.float64, n_aux * n_bf * n_bf),
                                          prec, _ptr(out, "out", torch.uint8, nbytes)))
        return out

    def build(self, b, C, H, occ, pair_of, n_pairs, n_cwo, prec=FP64, functional=PNOF7, out=None, b_split=None):
        """Transform, J/K (MO), J^q/K^q (AO), energy, Lagrangian and gradient in
        one rif_build call.  `out` (a dict from a previous call with the same
        shapes) is reused to avoid allocations; `b_split` is presplit_b's
        result for this `prec` (or None)."""
        n_aux, n_bf, _ = b.shape
        if out is None:
            out = self.outputs(n_bf, n_aux, n_pairs, n_cwo, C.shape[1], prec, b.device)
        inp = {"b": b, "C": C, "H": H, "occ": occ, "pair_of": pair_of, "b_split": b_split}
        inst = self.instance(inp, n_pairs, n_cwo, out, prec)
        self._chk(self.lib.rif_build(self.h, ctypes.byref(inst), prec, functional))
        return out

    def build_direct(self, b, C, H, occ, pair_of, n_pairs, n_cwo, prec=FP64, functional=PNOF7, out=None,
                     b_split=None):
        """rif_build_direct: energy, lambda and G without the per-MO AO
        matrices (out has no Jn/Kn)."""
        n_aux, n_bf, _ = b.shape
        if out is None:
            out = self.outputs(n_bf, n_aux, n_pairs, n_cwo, C.shape[1], prec, b.device, per_mo_ao=False)
        inp = {"b": b, "C": C, "H": H, "occ": occ, "pair_of": pair_of, "b_split": b_split}
        inst = self.instance(inp, n_pairs, n_cwo, out, prec)
        self._chk(self.lib.rif_build_direct(self.h, ctypes.byref(inst), prec, functional))
        return out

    def build_steps(self, b, C, H, occ, pair_of, n_pairs, n_cwo, prec=FP64, functional=PNOF7, out=None):
        """The same build as four ABI calls (rif_transform, rif_jk_mo,
        rif_jk_ao_per_mo, pnof_energy_grad) on one stream."""
        n_omega = n_pairs * (1 + n_cwo)
        o = out if out is not None else {}
        o["b_half"], o["b_mo"], o["d"] = self.transform(b, C, n_omega, prec, o.get("b_half"),
                                                        o.get("b_mo"), o.get("d"))
        o["J"], o["K"] = self.jk_mo(o["b_mo"], o["d"], prec, o.get("J"), o.get("K"))
        o["Jn"], o["Kn"] = self.jk_ao_per_mo(b, o["b_half"], o["d"], prec, o.get("Jn"), o.get("Kn"))
        o["energy"], o["lam"], o["grad"] = self.energy_grad(
            H, C, occ, pair_of, n_pairs, n_cwo, o["J"], o["K"], o["Jn"], o["Kn"], prec, functional,
            o.get("energy"), o.get("lam"), o.get("grad"))
        return o

    # ---- instances and batches ---------------------------------------------
    def outputs(self, n_bf, n_aux, n_pairs, n_cwo, n_mo, prec=FP64, device="cuda", per_mo_ao=True):
        """Allocate every output array of one build (without Jn/Kn if not
        per_mo_ao)."""
        import torch
        w = n_pairs * (1 + n_cwo)
        dt = torch.float64 if prec == FP64 else torch.float32
        f64 = torch.float64
        return {"b_half": torch.empty((w, n_aux, n_bf), dtype=dt, device=device),
                "b_mo": torch.empty((n_aux, w, w), dtype=dt, device=device),
                "d": torch.empty((n_aux, w), dtype=f64, device=device),
                "J": torch.empty((w, w), dtype=f64, device=device),
                "K": torch.empty((w, w), dtype=f64, device=device),
                "Jn": torch.empty((w, n_bf, n_bf), dtype=dt, device=device) if per_mo_ao else None,
                "Kn": torch.empty((w, n_bf, n_bf), dtype=dt, device=device) if per_mo_ao else None,
                "energy": torch.empty((1,), dtype=f64, device=device),
                "lam": torch.empty((n_mo, w), dtype=f64, device=device),
                "grad": torch.empty((n_mo, n_mo), dtype=f64, device=device)}

    @staticmethod
    def instance(inp, n_pairs, n_cwo, out, prec=FP64):
        """rif_instance from input tensors (b, C, H, occ, pair_of) and outputs."""
        import torch
        n_aux, n_bf, _ = inp["b"].shape
        n_mo = inp["C"].shape[1]
        w = n_pairs * (1 + n_cwo)
        dt = torch.float64 if prec == FP64 else torch.float32
        f64 = torch.float64
        return Instance(
            n_bf, n_aux, n_pairs, n_cwo, n_mo,
            _ptr(inp["b"], "b", f64, n_aux * n_bf * n_bf), _ptr(inp["C"], "C", f64, n_bf * n_mo),
            _ptr(inp["H"], "H", f64, n_bf * n_bf), _ptr(inp["occ"], "occ", f64, w),
            _ptr(inp.get("pair_of"), "pair_of", torch.int32, w),
            _ptr(out["b_half"], "b_half", dt, w * n_aux * n_bf), _ptr(out["b_mo"], "b_mo", dt, n_aux * w * w),
            _ptr(out["d"], "d", f64, n_aux * w), _ptr(out["J"], "J", f64, w * w), _ptr(out["K"], "K", f64, w * w),
            _ptr(out.get("Jn"), "Jn", dt, w * n_bf * n_bf), _ptr(out.get("Kn"), "Kn", dt, w * n_bf * n_bf),
            _ptr(out["energy"], "energy", f64, 1), _ptr(out["lam"], "lambda", f64, n_mo * w),
            _ptr(out["grad"], "grad", f64, n_mo * n_mo), _ptr(inp.get("b_split"), "b_split", torch.uint8))

    def build_instance(self, inp, n_pairs, n_cwo, out=None, prec=FP64, functional=PNOF7):
        """One build through rif_build."""
        n_aux, n_bf, _ = inp["b"].shape
        if out is None:
            out = self.outputs(n_bf, n_aux, n_pairs, n_cwo, inp["C"].shape[1], prec, inp["b"].device)
        inst = self.instance(inp, n_pairs, n_cwo, out, prec)
        self._chk(self.lib.rif_build(self.h, ctypes.byref(inst), prec, functional))
        return out

    def batch(self, items, prec=FP64, functional=PNOF7):
        """items: list of (inputs dict, n_pairs, n_cwo, outputs dict or None)."""
        return Batch(self, items, prec, functional)

    # ---- ON optimisation and the warm-start MLP ----------------------------
    def hpp(self, H, C, n_omega, out=None):
        import torch
        n_bf, n_mo = C.shape
        out = torch.empty(n_omega, dtype=torch.float64, device=C.device) if out is None else out
        self._chk(self.lib.rif_hpp(self.h, n_bf, n_mo, n_omega, _ptr(H, "H", torch.float64, n_bf * n_bf),
                                   _ptr(C, "C", torch.float64, n_bf * n_mo), _ptr(out, "Hpp", torch.float64, n_omega)))
        return out

    def on_optimize(self, onset):
        self._chk(self.lib.rif_on_optimize(self.h, len(onset.arr), onset.arr))

    def on_features(self, onset, X, T=None, M=None, mu=None, sigma=None):
        import torch
        f32 = torch.float32
        self._chk(self.lib.rif_on_features(
            self.h, len(onset.arr), onset.arr, _ptr(X, "X", f32, onset.rows * 39),
            _ptr(T, "T", f32, onset.rows * 7), _ptr(M, "M", f32, onset.rows * 7),
            _ptr(mu, "mu", f32, 39), _ptr(sigma, "sigma", f32, 39)))

    def on_warmstart(self, onset, P):
        import torch
        self._chk(self.lib.rif_on_warmstart(self.h, len(onset.arr), onset.arr,
                                            _ptr(P, "P", torch.float32, onset.rows * 7)))

    # ---- b from the three-centre integrals and the metric --------------------
    def prepare_b(self, T, G, delta=0.0, b=None, factors=False):
        """rif_prepare_b: b [n_aux][n_bf][n_bf].  With factors=True also
        returns perm, L, D (dense) and the number of raised eigenvalues."""
        import torch
        n_aux, n_bf, _ = T.shape
        if b is None:
            b = torch.empty_like(T)
        perm = L = D = nr = None
        if factors:
            perm = torch.empty(n_aux, dtype=torch.int32, device=T.device)
            L = torch.empty((n_aux, n_aux), dtype=torch.float64, device=T.device)
            D = torch.empty((n_aux, n_aux), dtype=torch.float64, device=T.device)
            nr = torch.zeros(1, dtype=torch.int32, device=T.device)
        self._chk(self.lib.rif_prepare_b(
            self.h, n_bf, n_aux, _ptr(T, "T", torch.float64, n_aux * n_bf * n_bf),
            _ptr(G, "G", torch.float64, n_aux * n_aux), float(delta), _ptr(b, "b", torch.float64, b.numel()),
            _ptr(perm, "perm", torch.int32, n_aux), _ptr(L, "L", torch.float64, n_aux * n_aux),
            _ptr(D, "D", torch.float64, n_aux * n_aux), _ptr(nr, "n_raised", torch.int32, 1)))
        return (b, perm, L, D, nr) if factors else b

    # ---- orbital optimisation and the outer/inner loop ----------------------
    def set_wait_limit(self, polls=1 << 22):
        """rif_set_wait_limit: polls of one exchanged value before the one-launch
        kernels give up (negative: at once)."""
        self._chk(self.lib.rif_set_wait_limit(self.h, int(polls)))

    def set_eigensolver(self, kind=EIG_AUTO, groups=0):
        """rif_set_eigensolver: EIG_DC (one-launch tridiagonal reduction, then the
        library's divide and conquer), EIG_TRD (the same reduction, then
        rocSOLVER dstedc), EIG_SYEVD (rocSOLVER dsyevd) or EIG_AUTO (DC where
        it fits, else SYEVD)."""
        self._chk(self.lib.rif_set_eigensolver(self.h, int(kind), int(groups)))

    def orbital_step(self, lam, C, n_omega, eps_in=None, eps_out=None, info=None):
        """One rif_orbital_step: C (in place) <- C V; returns eps_out."""
        import torch
        n_bf, n_mo = C.shape
        if eps_out is None:
            eps_out = torch.empty(n_mo, dtype=torch.float64, device=C.device)
        self._chk(self.lib.rif_orbital_step(
            self.h, n_bf, n_mo, n_omega, _ptr(lam, "lambda", torch.float64, n_mo * n_omega),
            _ptr(eps_in, "eps_in", torch.float64, n_mo), _ptr(C, "C", torch.float64, n_bf * n_mo),
            _ptr(eps_out, "eps_out", torch.float64, n_mo), _ptr(info, "info", torch.int32, 1)))
        return eps_out

    def optimize(self, b, C, H, occ, gamma, pair_of, n_pairs, n_cwo, prec=FP64, functional=PNOF7,
                 max_outer=50, max_inner=500, on_max_it=2000, tol_grad=1e-8, tol_energy=1e-10, on_tol=1e-10,
                 init_gamma=0, hist_len=0, out=None, direct=True):
        """rif_pnof_optimize: C, occ and gamma are updated in place.  Returns
        (result dict, per-inner-iteration energies, max|G|) with the histories
        as lists of at most hist_len entries.  direct: inner builds without
        the per-MO AO matrices (no Jn/Kn buffers)."""
        n_aux, n_bf, _ = b.shape
        if out is None:
            out = self.outputs(n_bf, n_aux, n_pairs, n_cwo, C.shape[1], prec, b.device, per_mo_ao=not direct)
        inp = {"b": b, "C": C, "H": H, "occ": occ, "pair_of": pair_of}
        inst = self.instance(inp, n_pairs, n_cwo, out, prec)
        import torch
        _ptr(gamma, "gamma", torch.float64, n_pairs * n_cwo)
        par = OptParams(max_outer, max_inner, on_max_it, init_gamma, tol_grad, tol_energy, on_tol)
        res = OptResult()
        he = (ctypes.c_double * max(hist_len, 1))()
        hg = (ctypes.c_double * max(hist_len, 1))()
        self._chk(self.lib.rif_pnof_optimize(
            self.h, ctypes.byref(inst), prec, functional, ctypes.byref(par), inst.C, inst.occ,
            ctypes.c_void_p(gamma.data_ptr()), ctypes.byref(res), he, hg, hist_len))
        n = min(hist_len, res.inner_total)
        return res.as_dict(), list(he[:n]), list(hg[:n])

    def mlp_n_params(self) -> int:
        return int(self.lib.rif_mlp_n_params())

    def mlp_forward(self, X, M, theta, H, Z, P):
        import torch
        f = torch.float32
        n = X.shape[0]
        self._chk(self.lib.rif_mlp_forward(self.h, n, _ptr(X, "X", f, n * 39), _ptr(M, "M", f, n * 7),
                                           _ptr(theta, "theta", f), _ptr(H, "H", f, 3 * n * 128),
                                           _ptr(Z, "Z", f, n * 7), _ptr(P, "P", f, n * 7)))

    def mlp_backward(self, X, M, T, theta, H, Z, dA, grad, loss):
        import torch
        f = torch.float32
        n = X.shape[0]
        self._chk(self.lib.rif_mlp_backward(
            self.h, n, _ptr(X, "X", f, n * 39), _ptr(M, "M", f, n * 7), _ptr(T, "T", f, n * 7),
            _ptr(theta, "theta", f), _ptr(H, "H", f, 3 * n * 128), _ptr(Z, "Z", f, n * 7),
            _ptr(dA, "dA", f, 2 * n * 128), _ptr(grad, "grad", f), _ptr(loss, "loss", torch.float64, 1)))

    def adam(self, theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        import torch
        f = torch.float32
        n = theta.numel()
        self._chk(self.lib.rif_adam(self.h, n, _ptr(theta, "theta", f, n), _ptr(grad, "grad", f, n),
                                    _ptr(m, "m", f, n), _ptr(v, "v", f, n), step, lr, beta1, beta2, eps))

    # ---- tile selection ---------------------------------------------------
    def autotune(self, on: bool = True):
        self._chk(self.lib.rif_autotune(self.h, 1 if on else 0))

    def set_tile_variant(self, v: int):
        self._chk(self.lib.rif_set_tile_variant(self.h, v))

    def tune_report(self) -> str:
        buf = ctypes.create_string_buffer(1 << 16)
        self._chk(self.lib.rif_tune_report(self.h, buf, len(buf)))
        return buf.value.decode()

    def tune_load(self, text: str):
        """rif_tune_load: tile choices from an earlier tune_report()."""
        self._chk(self.lib.rif_tune_load(self.h, text.encode()))

    # ---- per-kernel timing ------------------------------------------------
    def profile(self, on: bool = True, only: str | None = None):
        """Start (or stop) per-launch event timing; `only` restricts it to
        launches of that report name."""
        self._chk(self.lib.rif_profile_only(self.h, only.encode() if only else None))
        self._chk(self.lib.rif_profile_enable(self.h, 1 if on else 0))

    def profile_report(self) -> dict:
        buf = ctypes.create_string_buffer(1 << 16)
        self._chk(self.lib.rif_profile_report(self.h, buf, len(buf)))
        out = {}
        for line in buf.value.decode().splitlines():
            name, n, ms = line.split()
            out[name] = (int(n), float(ms))
        return out


class Batch:
    """A rif_batch: many molecules built by one grouped launch per step."""

    def __init__(self, ctx: Context, items, prec=FP64, functional=PNOF7):
        self.ctx = ctx
        self.outs, self.inputs = [], []
        arr = (Instance * len(items))()
        for i, (inp, n_pairs, n_cwo, out) in enumerate(items):
            n_aux, n_bf, _ = inp["b"].shape
            if out is None:
                out = ctx.outputs(n_bf, n_aux, n_pairs, n_cwo, inp["C"].shape[1], prec, inp["b"].device)
            self.inputs.append(inp)
            self.outs.append(out)
            arr[i] = Context.instance(inp, n_pairs, n_cwo, out, prec)
        h = ctypes.c_void_p()
        ctx._chk(ctx.lib.rif_batch_create(ctx.h, len(items), arr, prec, functional, ctypes.byref(h)))
        self.h = h
        _live_batches.add(self)

    def run(self, use_graph: bool = True):
        self.ctx._chk(self.ctx.lib.rif_batch_run(self.h, 1 if use_graph else 0))

    def close(self):
        if getattr(self, "h", None):
            if getattr(self.ctx, "h", None):
                self.ctx.lib.rif_batch_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class OnSet:
    """A set of ON-optimisation problems (one per molecule) with their device
    buffers: gamma, occ, energy, iters, status and work.  `problems` is a list
    of (Hpp, J, K, pair_of or None, n_pairs, n_cwo) device tensors/ints."""

    def __init__(self, lib_ctx: Context, problems, tol=1e-8, max_it=2000, functional=PNOF7, device="cuda"):
        import torch
        self.ctx = lib_ctx
        n = len(problems)
        self.keep = []
        self.arr = (OnProblem * n)()
        self.rows = 0
        sizes = [(p[4], p[5]) for p in problems]
        nv = [a * b for a, b in sizes]
        self.gamma = torch.zeros(sum(nv), dtype=torch.float64, device=device)
        self.occ = torch.zeros(sum(a * (1 + b) for a, b in sizes), dtype=torch.float64, device=device)
        self.energy = torch.zeros(n, dtype=torch.float64, device=device)
        self.iters = torch.zeros(n, dtype=torch.int32, device=device)
        self.status = torch.zeros(n, dtype=torch.int32, device=device)
        ws = [int(lib_ctx.lib.rif_on_work_size(a * (1 + b), a, b)) for a, b in sizes]
        self.work = torch.zeros(sum(ws), dtype=torch.float64, device=device)
        self.gslices, self.oslices = [], []
        go = oo = wo = 0
        for i, (Hpp, J, K, pm, npair, ncwo) in enumerate(problems):
            w = npair * (1 + ncwo)
            q = self.arr[i]
            q.n_pairs, q.n_cwo, q.n_omega, q.functional, q.max_it, q.row0 = npair, ncwo, w, functional, max_it, self.rows
            q.tol = tol
            q.Hpp = _ptr(Hpp, "Hpp", torch.float64, w)
            q.J = _ptr(J, "J", torch.float64, w * w)
            q.K = _ptr(K, "K", torch.float64, w * w)
            q.pair_of = _ptr(pm, "pair_of", torch.int32, w) if pm is not None else None
            q.gamma = self.gamma.data_ptr() + 8 * go
            q.occ = self.occ.data_ptr() + 8 * oo
            q.energy = self.energy.data_ptr() + 8 * i
            q.iters = self.iters.data_ptr() + 4 * i
            q.status = self.status.data_ptr() + 4 * i
            q.work = self.work.data_ptr() + 8 * wo
            self.keep.append((Hpp, J, K, pm))
            self.gslices.append(slice(go, go + npair * ncwo))
            self.oslices.append(slice(oo, oo + w))
            go += npair * ncwo
            oo += w
            wo += ws[i]
            self.rows += npair
        self.sizes = sizes
