"""ctypes binding of libkmx (include/kmx.h).

Argument marshalling only: every tensor must already live on the GPU; torch
supplies device memory and the current stream, and every step of the
computation runs in the library's HIP kernels.  Calls raise ``KmxError`` when
the library reports a failure, and ``RuntimeError`` when the library is not
built -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import weakref
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkmx.so")

FP32, BF16, FP8 = 0, 1, 2
_PREC = {"fp32": FP32, "bf16": BF16, "fp8": FP8, FP32: FP32, BF16: BF16, FP8: FP8}

TIMING_CLASSES = ("prep", "assign", "recheck", "sort", "reduce", "finalize", "seed", "other",
                  "router", "certificate", "train", "project", "bounds", "short_recheck")
ROUTER_HIDDEN = 256
ROUTER_M = 16

_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


class Problem(ctypes.Structure):
    """kmx_problem: one instance of a batched call (device pointers)."""
    _fields_ = [("X", ctypes.c_void_p), ("n", ctypes.c_int64), ("d", ctypes.c_int32),
                ("ldx", ctypes.c_int64), ("w", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("k", ctypes.c_int32), ("label", ctypes.c_void_p)]


class KmxError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"kmx status {status}: {message}")
        self.status = status


def lib():
    """Loads libkmx.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1502_04265_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "kmx_create": [ctypes.POINTER(_vp), ctypes.c_int, _vp],
        "kmx_destroy": [_vp],
        "kmx_set_stream": [_vp, _vp],
        "kmx_invalidate": [_vp, _vp],
        "kmx_seed": [_vp, _vp, _i64, _i32, _i64, _vp, _i32, ctypes.c_uint64, _vp, _vp],
        "kmx_assign": [_vp, _vp, _i64, _i32, _i64, _vp, _i32, ctypes.c_int, _vp, _vp, _vp, _vp],
        "kmx_assign_noalloc": [_vp, _vp, _i64, _i32, _i64, _vp, _i32, _vp, _vp, _vp],
        "kmx_update": [_vp, _vp, _i64, _i32, _i64, _vp, _vp, _i32, _vp, _vp, _vp, _vp],
        "kmx_cost": [_vp, _vp, _i64, _i32, _i64, _vp, _vp, _i32, ctypes.c_int, _vp],
        "kmx_lloyd": [_vp, _vp, _i64, _i32, _i64, _vp, _vp, _i32, _i32, ctypes.c_double,
                      ctypes.c_int, _vp, _vp, _vp],
        "kmx_lloyd_graph": [_vp, _vp, _i64, _i32, _i64, _vp, _vp, _i32, _i32, ctypes.c_double,
                            ctypes.c_int, _vp, _vp, _vp],
        "kmx_timing": [_vp, ctypes.c_int, ctypes.c_int],
        "kmx_mfma_probe": [_vp, ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _i32],
        "kmx_assign_stats": [_vp, _vp, _vp, _vp],
        "kmx_update_stats": [_vp, _vp, _vp],
        "kmx_run_stats": [_vp, _vp, _vp],
        "kmx_seed_stats": [_vp, _vp],
        "kmx_timing_read": [_vp, ctypes.c_int, _vp, _vp],
        "kmx_lloyd_batched": [_vp, _vp, _i32, _i32, ctypes.c_int, _vp],
        "kmx_seed_batched": [_vp, _vp, _i32, _vp, _vp],
        "kmx_batched_autotune": [_vp, _vp, _i32, ctypes.c_int, ctypes.c_char_p, _vp],
        "kmx_batched_tiles": [_vp, _i32, _i32, _vp, _vp],
        "kmx_project": [_vp, _vp, _i64, _i32, _i64, _vp, _i32, _vp, _i64],
        "kmx_lift": [_vp, _vp, _i64, _i32, _i64, _vp, _i32, _vp, _i64],
        "kmx_range_basis": [_vp, _vp, _i64, _i32, _i64, _vp, _i32, _i32, _i32, ctypes.c_uint64,
                            _vp, _vp],
        "kmx_router_create": [_vp, _i32, _i32, ctypes.c_uint64, ctypes.POINTER(_vp)],
        "kmx_router_destroy": [_vp, _vp],
        "kmx_router_set_params": [_vp, _vp, _vp, _vp, _vp, _vp],
        "kmx_router_get_params": [_vp, _vp, _vp, _vp, _vp, _vp],
        "kmx_router_loss_grad": [_vp, _vp, _vp, _i64, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp],
        "kmx_router_train": [_vp, _vp, _vp, _i64, _i32, _i64, _vp, _i32, _i32, _i32,
                             ctypes.c_float, ctypes.c_uint64, _vp, _vp],
        "kmx_router_propose": [_vp, _vp, _vp, _i64, _i32, _i64, _vp],
        "kmx_center_bounds": [_vp, _vp, _i32, _i32, _vp],
        "kmx_lloyd_routed": [_vp, _vp, _vp, _i64, _i32, _i64, _vp, _vp, _i32, _i32,
                             ctypes.c_double, ctypes.c_int, _vp, _vp, _vp, _vp],
        "kmx_lloyd_bounded": [_vp, _vp, _vp, _i64, _i32, _i64, _vp, _vp, _i32, _i32,
                              ctypes.c_double, ctypes.c_int, _vp, _vp, _vp, _vp, _vp],
        "kmx_bico_create": [_vp, _i32, _i64, ctypes.c_double, ctypes.POINTER(_vp)],
        "kmx_bico_destroy": [_vp, _vp],
        "kmx_bico_insert": [_vp, _vp, _vp, _i64, _i64, _vp],
        "kmx_bico_stats": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
        "kmx_bico_features": [_vp, _vp, _vp, _vp, _vp, _vp, _vp],
        "kmx_bico_coreset": [_vp, _vp, _vp, _vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.kmx_last_error.argtypes = [_vp]
    L.kmx_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status: int, ctx_ptr) -> None:
    if status != 0:
        msg = lib().kmx_last_error(ctx_ptr)
        raise KmxError(status, msg.decode() if msg else "")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else _vp(t.data_ptr())


def _rows(X: torch.Tensor):
    if not X.is_cuda or X.dtype != torch.float32 or X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be a 2-D float32 CUDA tensor with unit column stride")
    return X.shape[0], X.shape[1], X.stride(0)


def _vec(w: Optional[torch.Tensor], n: int, dtype=torch.float32):
    if w is None:
        return None
    if not w.is_cuda or w.dtype != dtype or w.numel() != n or not w.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} CUDA tensor of {n} elements")
    return w


def _centers(C: torch.Tensor, d: int):
    if not C.is_cuda or C.dtype != torch.float32 or C.dim() != 2 or C.shape[1] != d \
            or not C.is_contiguous():
        raise ValueError("C must be a contiguous k x d float32 CUDA tensor")
    return C.shape[0]


class Context:
    """Owns a kmx_ctx bound to one device; every call runs on torch's current
    stream of that device."""

    def __init__(self, device: int = 0):
        L = lib()
        self.device = int(device)
        p = _vp()
        with torch.cuda.device(self.device):
            st = torch.cuda.current_stream().cuda_stream
            _check(L.kmx_create(ctypes.byref(p), self.device, _vp(st)), None)
        self._p = p
        self._xseen = {}

    def _fresh(self, X):
        """The library caches derived copies of X by device pointer.  A
        different tensor at a pointer seen before (the old one freed and its
        memory reused), or an in-place change of the same tensor (its version
        counter moved), drops that cache first."""
        key = X.data_ptr()
        seen = self._xseen.get(key)
        if seen is not None and (seen[0]() is not X or seen[1] != X._version):
            _check(lib().kmx_invalidate(self._p, _vp(key)), self._p)
        self._xseen[key] = (weakref.ref(X), X._version)

    def close(self):
        if getattr(self, "_p", None) is not None and self._p.value:
            lib().kmx_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        st = torch.cuda.current_stream(self.device).cuda_stream
        lib().kmx_set_stream(self._p, _vp(st))

    # ---- the five calls ----------------------------------------------------
    def seed(self, X, k: int, w=None, rng_seed: int = 0):
        n, d, ldx = _rows(X)
        _vec(w, n)
        C = torch.empty((k, d), dtype=torch.float32, device=X.device)
        idx = torch.empty(k, dtype=torch.int64, device=X.device)
        self._sync_stream()
        _check(lib().kmx_seed(self._p, _ptr(X), n, d, ldx, _ptr(w), k,
                              ctypes.c_uint64(rng_seed & (2 ** 64 - 1)), _ptr(C), _ptr(idx)),
               self._p)
        return C, idx

    def assign(self, X, C, prec="fp32", want_d=True):
        n, d, ldx = _rows(X)
        self._fresh(X)
        k = _centers(C, d)
        lab = torch.empty(n, dtype=torch.int32, device=X.device)
        d1 = torch.empty(n, dtype=torch.float32, device=X.device) if want_d else None
        d2 = torch.empty(n, dtype=torch.float32, device=X.device) if want_d else None
        nf = ctypes.c_int64(0)
        self._sync_stream()
        _check(lib().kmx_assign(self._p, _ptr(X), n, d, ldx, _ptr(C), k, _PREC[prec], _ptr(lab),
                                _ptr(d1), _ptr(d2), ctypes.byref(nf)), self._p)
        return lab, d1, d2, int(nf.value)

    def assign_noalloc(self, X, C, label, d1=None, d2=None):
        """kmx_assign_noalloc: the FP32 assignment into caller-provided outputs,
        with no device allocation inside the library."""
        n, d, ldx = _rows(X)
        k = _centers(C, d)
        _vec(label, n, torch.int32)
        _vec(d1, n)
        _vec(d2, n)
        self._sync_stream()
        _check(lib().kmx_assign_noalloc(self._p, _ptr(X), n, d, ldx, _ptr(C), k, _ptr(label),
                                        _ptr(d1), _ptr(d2)), self._p)

    def update(self, X, labels, C_prev, w=None, out=None):
        n, d, ldx = _rows(X)
        k = _centers(C_prev, d)
        _vec(labels, n, torch.int32)
        _vec(w, n)
        C_out = torch.empty_like(C_prev) if out is None else out
        W = torch.empty(k, dtype=torch.float64, device=X.device)
        cac = ctypes.c_double(0.0)
        self._sync_stream()
        _check(lib().kmx_update(self._p, _ptr(X), n, d, ldx, _ptr(w), _ptr(labels), k,
                                _ptr(C_prev), _ptr(C_out), _ptr(W), ctypes.byref(cac)), self._p)
        return C_out, W, float(cac.value)

    def cost(self, X, C, w=None, prec="fp32") -> float:
        n, d, ldx = _rows(X)
        self._fresh(X)
        k = _centers(C, d)
        _vec(w, n)
        out = ctypes.c_double(0.0)
        self._sync_stream()
        _check(lib().kmx_cost(self._p, _ptr(X), n, d, ldx, _ptr(w), _ptr(C), k, _PREC[prec],
                              ctypes.byref(out)), self._p)
        return float(out.value)

    def lloyd(self, X, C0, max_iter: int, w=None, tol: float = -1.0, prec="bf16",
              labels: bool = True, inplace: bool = False, graph: bool = False):
        """kmx_lloyd, or kmx_lloyd_graph with graph=True (one captured
        iteration replayed); returns (C, labels, cost_hist, iters)."""
        n, d, ldx = _rows(X)
        self._fresh(X)
        k = _centers(C0, d)
        _vec(w, n)
        C = C0 if inplace else C0.clone()
        lab = torch.empty(n, dtype=torch.int32, device=X.device) if labels else None
        hist = (ctypes.c_double * (max_iter + 1))()
        iters = ctypes.c_int32(0)
        self._sync_stream()
        fn = lib().kmx_lloyd_graph if graph else lib().kmx_lloyd
        _check(fn(self._p, _ptr(X), n, d, ldx, _ptr(w), _ptr(C), k, max_iter, float(tol),
                  _PREC[prec], _ptr(lab), hist, ctypes.byref(iters)), self._p)
        it = int(iters.value)
        return C, lab, [hist[i] for i in range(it + 1)], it

    def invalidate(self, X=None):
        _check(lib().kmx_invalidate(self._p, _ptr(X)), self._p)

    # ---- measurement -------------------------------------------------------
    def seed_stats(self):
        """Rows whose distance the most recent seed() computed (rounds 1 .. k-1)."""
        a = ctypes.c_int64(0)
        _check(lib().kmx_seed_stats(self._p, ctypes.byref(a)), self._p)
        return int(a.value)

    def assign_stats(self):
        """(listed, fp32, full) re-check counts of the most recent assignment."""
        a, b, c = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
        _check(lib().kmx_assign_stats(self._p, ctypes.byref(a), ctypes.byref(b),
                                      ctypes.byref(c)), self._p)
        return int(a.value), int(b.value), int(c.value)

    def run_stats(self):
        """(listed_total, full_total): short re-check entries and every-center
        rows summed over the assignments of the most recent Lloyd run."""
        a, b = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(lib().kmx_run_stats(self._p, ctypes.byref(a), ctypes.byref(b)), self._p)
        return int(a.value), int(b.value)

    def update_stats(self):
        """(changed, delta) of the most recent update of a Lloyd run: the rows
        whose label changed and whether the delta path formed the features."""
        a, b = ctypes.c_int64(0), ctypes.c_int32(0)
        _check(lib().kmx_update_stats(self._p, ctypes.byref(a), ctypes.byref(b)), self._p)
        return int(a.value), bool(b.value)

    def mfma_probe(self, prec, A, B, scale_a=None, scale_b=None, C=None):
        """kmx_mfma_probe.  A, B: (count, 16, K) uint8 E4M3 bytes (fp8, K = 128),
        int16 BF16 bit patterns (bf16, K = 32) or float32 (fp32, K = 4); fp8
        scales uint8 (count,) and (count, 16); optional start values C float32
        (count, 16, 16).  Returns D (count, 16, 16)."""
        p = _PREC[prec]
        kk, dt = {FP8: (128, torch.uint8), BF16: (32, torch.int16), FP32: (4, torch.float32)}[p]
        count = A.shape[0]
        for t, shape in ((A, (count, 16, kk)), (B, (count, 16, kk))):
            if not t.is_cuda or t.dtype != dt or tuple(t.shape) != shape or not t.is_contiguous():
                raise ValueError(f"expected a contiguous {dt} CUDA tensor of shape {shape}")
        if p == FP8:
            for t, shape in ((scale_a, (count,)), (scale_b, (count, 16))):
                if t is None or not t.is_cuda or t.dtype != torch.uint8 \
                        or tuple(t.shape) != shape or not t.is_contiguous():
                    raise ValueError(f"expected a contiguous uint8 CUDA tensor of shape {shape}")
        if C is not None and (not C.is_cuda or C.dtype != torch.float32
                              or tuple(C.shape) != (count, 16, 16) or not C.is_contiguous()):
            raise ValueError("C must be a contiguous float32 CUDA tensor (count, 16, 16)")
        D = torch.empty((count, 16, 16), dtype=torch.float32, device=A.device)
        self._sync_stream()
        _check(lib().kmx_mfma_probe(self._p, p, _ptr(A), _ptr(B), _ptr(scale_a), _ptr(scale_b),
                                    _ptr(C), _ptr(D), count), self._p)
        return D

    def timing(self, enable: bool = True, reset: bool = True):
        _check(lib().kmx_timing(self._p, int(enable), int(reset)), self._p)

    def timing_read(self):
        nc = len(TIMING_CLASSES)
        ms = (ctypes.c_double * nc)()
        cnt = (ctypes.c_int64 * nc)()
        _check(lib().kmx_timing_read(self._p, nc, ms, cnt), self._p)
        return {name: (ms[i], cnt[i]) for i, name in enumerate(TIMING_CLASSES)}

    # ---- batched instances ----------------------------------------------------
    def _problems(self, problems, labels=True, inplace=False):
        arr = (Problem * len(problems))()
        keep = []
        for i, p in enumerate(problems):
            X, C0 = p["X"], p["C"]
            w = p.get("w")
            n, d, ldx = _rows(X)
            k = _centers(C0, d)
            _vec(w, n)
            self._fresh(X)
            if w is not None:
                self._fresh(w)
            C = C0 if inplace else C0.clone()
            lab = torch.empty(n, dtype=torch.int32, device=X.device) if labels else None
            keep.append((C, lab))
            arr[i] = Problem(X.data_ptr(), n, d, ldx, w.data_ptr() if w is not None else None,
                             C.data_ptr(), k, lab.data_ptr() if lab is not None else None)
        return arr, keep

    def lloyd_batched(self, problems, iters: int, prec="bf16", labels: bool = True,
                      inplace: bool = False):
        """problems: list of dicts with X (n x d), C (k x d initial centers), optional w.
        Returns [(C, labels, cost_hist)] in the same order."""
        arr, keep = self._problems(problems, labels, inplace)
        hist = (ctypes.c_double * (len(problems) * (iters + 1)))()
        self._sync_stream()
        _check(lib().kmx_lloyd_batched(self._p, arr, len(problems), iters, _PREC[prec], hist),
               self._p)
        s = iters + 1
        return [(keep[i][0], keep[i][1], [hist[i * s + t] for t in range(s)])
                for i in range(len(problems))]

    def seed_batched(self, problems, rng_seeds):
        """kmx_seed_batched: problems are dicts with X (n x d), k, optional w;
        returns [(C, idx)] in the same order."""
        arr = (Problem * len(problems))()
        keep = []
        for i, p in enumerate(problems):
            X, k, w = p["X"], int(p["k"]), p.get("w")
            n, d, ldx = _rows(X)
            _vec(w, n)
            C = torch.empty((k, d), dtype=torch.float32, device=X.device)
            keep.append(C)
            arr[i] = Problem(X.data_ptr(), n, d, ldx, w.data_ptr() if w is not None else None,
                             C.data_ptr(), k, None)
        ks = [int(p["k"]) for p in problems]
        idx = torch.empty(sum(ks), dtype=torch.int64, device=problems[0]["X"].device)
        seeds = (ctypes.c_uint64 * len(problems))(*[int(v) & (2 ** 64 - 1) for v in rng_seeds])
        self._sync_stream()
        _check(lib().kmx_seed_batched(self._p, arr, len(problems), seeds, _ptr(idx)), self._p)
        out, o = [], 0
        for C, k in zip(keep, ks):
            out.append((C, idx[o:o + k]))
            o += k
        return out

    def batched_autotune(self, problems, cache_path=None, prec="bf16"):
        """Tile shapes for the batched assignment; returns True when read from the cache."""
        arr, _ = self._problems(problems, labels=False)
        loaded = ctypes.c_int32(0)
        self._sync_stream()
        _check(lib().kmx_batched_autotune(self._p, arr, len(problems), _PREC[prec],
                                          cache_path.encode() if cache_path else None,
                                          ctypes.byref(loaded)), self._p)
        return bool(loaded.value)

    def batched_tiles(self, d: int, k: int):
        t, p = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().kmx_batched_tiles(self._p, d, k, ctypes.byref(t), ctypes.byref(p)), self._p)
        return int(t.value), int(p.value)

    def project(self, X, V, out=None):
        """Y = X V for a chunk of rows (kmx_project); V is d_in x d_out float32."""
        rows, d_in, ldx = _rows(X)
        if not V.is_cuda or V.dtype != torch.float32 or V.dim() != 2 or V.shape[0] != d_in \
                or not V.is_contiguous():
            raise ValueError("V must be a contiguous d_in x d_out float32 CUDA tensor")
        d_out = V.shape[1]
        Y = torch.empty((rows, d_out), dtype=torch.float32, device=X.device) if out is None else out
        self._sync_stream()
        _check(lib().kmx_project(self._p, _ptr(X), rows, d_in, ldx, _ptr(V), d_out, _ptr(Y),
                                 Y.stride(0)), self._p)
        return Y

    def lift(self, Z, V, out=None):
        """Y = Z V^T (kmx_lift): coordinates Z (rows x m) in the basis V (d x m)
        back to R^d."""
        rows, m, ldz = _rows(Z)
        if not V.is_cuda or V.dtype != torch.float32 or V.dim() != 2 or V.shape[1] != m \
                or not V.is_contiguous():
            raise ValueError("V must be a contiguous d x m float32 CUDA tensor")
        d = V.shape[0]
        Y = torch.empty((rows, d), dtype=torch.float32, device=Z.device) if out is None else out
        self._sync_stream()
        _check(lib().kmx_lift(self._p, _ptr(Z), rows, m, ldz, _ptr(V), d, _ptr(Y), Y.stride(0)),
               self._p)
        return Y

    def center_bounds(self, C):
        """kmx_center_bounds: k x k lower bounds of the distances between the
        rows of C (+inf on the diagonal)."""
        if not C.is_cuda or C.dtype != torch.float32 or C.dim() != 2 or not C.is_contiguous():
            raise ValueError("C must be a contiguous k x d float32 CUDA tensor")
        k, d = C.shape
        D = torch.empty((k, k), dtype=torch.float32, device=C.device)
        self._sync_stream()
        _check(lib().kmx_center_bounds(self._p, _ptr(C), k, d, _ptr(D)), self._p)
        return D

    def range_basis(self, A, r: int, w=None, oversample: int = 16, power_iters: int = 2,
                    seed: int = 0):
        """kmx_range_basis: the top-r right singular vectors of diag(sqrt w) A
        (d x r float32 CUDA tensor) and the singular values (list)."""
        n, d, lda = _rows(A)
        _vec(w, n)
        V = torch.empty((d, r), dtype=torch.float32, device=A.device)
        sig = (ctypes.c_double * r)()
        self._sync_stream()
        _check(lib().kmx_range_basis(self._p, _ptr(A), n, d, lda, _ptr(w), r, oversample,
                                     power_iters, ctypes.c_uint64(seed & (2 ** 64 - 1)), _ptr(V),
                                     sig), self._p)
        return V, [sig[i] for i in range(r)]

    # ---- candidate router ----------------------------------------------------
    def router(self, d: int, k: int, init_seed: int = 0) -> "Router":
        return Router(self, d, k, init_seed)

    def lloyd_routed(self, X, C0, max_iter: int, router: Optional["Router"] = None, w=None,
                     tol: float = -1.0, prec="bf16", labels: bool = True, inplace: bool = False):
        """kmx_lloyd_routed; returns (C, labels, cost_hist, iters, gemm_rows)."""
        n, d, ldx = _rows(X)
        self._fresh(X)
        k = _centers(C0, d)
        _vec(w, n)
        C = C0 if inplace else C0.clone()
        lab = torch.empty(n, dtype=torch.int32, device=X.device) if labels else None
        hist = (ctypes.c_double * (max_iter + 1))()
        rows = (ctypes.c_int64 * (max_iter + 1))()
        iters = ctypes.c_int32(0)
        self._sync_stream()
        _check(lib().kmx_lloyd_routed(self._p, router._r if router is not None else None,
                                      _ptr(X), n, d, ldx, _ptr(w), _ptr(C), k, max_iter,
                                      float(tol), _PREC[prec], _ptr(lab), hist,
                                      ctypes.byref(iters), rows), self._p)
        it = int(iters.value)
        return (C, lab, [hist[i] for i in range(it + 1)], it, [rows[i] for i in range(it + 1)])


    def lloyd_bounded(self, X, C0, max_iter: int, router: Optional["Router"] = None, w=None,
                      tol: float = -1.0, prec="bf16", labels: bool = True,
                      inplace: bool = False):
        """kmx_lloyd_bounded; returns (C, labels, cost_hist, iters, gemm_rows, kept_rows)."""
        n, d, ldx = _rows(X)
        self._fresh(X)
        k = _centers(C0, d)
        _vec(w, n)
        C = C0 if inplace else C0.clone()
        lab = torch.empty(n, dtype=torch.int32, device=X.device) if labels else None
        hist = (ctypes.c_double * (max_iter + 1))()
        rows = (ctypes.c_int64 * (max_iter + 1))()
        kept = (ctypes.c_int64 * (max_iter + 1))()
        iters = ctypes.c_int32(0)
        self._sync_stream()
        _check(lib().kmx_lloyd_bounded(self._p, router._r if router is not None else None,
                                       _ptr(X), n, d, ldx, _ptr(w), _ptr(C), k, max_iter,
                                       float(tol), _PREC[prec], _ptr(lab), hist,
                                       ctypes.byref(iters), rows, kept), self._p)
        it = int(iters.value)
        return (C, lab, [hist[i] for i in range(it + 1)], it, [rows[i] for i in range(it + 1)],
                [kept[i] for i in range(it + 1)])


class Router:
    """kmx_router: the candidate network (256 hidden units) for inputs of
    width d and k centers, with its FP32 parameters and Adam state on the
    device."""

    def __init__(self, ctx: Context, d: int, k: int, init_seed: int = 0):
        self.ctx = ctx
        self.d, self.k = int(d), int(k)
        r = _vp()
        _check(lib().kmx_router_create(ctx._p, self.d, self.k,
                                       ctypes.c_uint64(init_seed & (2 ** 64 - 1)),
                                       ctypes.byref(r)), ctx._p)
        self._r = r

    def close(self):
        if getattr(self, "_r", None) is not None and self._r.value:
            lib().kmx_router_destroy(self.ctx._p, self._r)
            self._r = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self):
        return torch.device("cuda", self.ctx.device)

    def get_params(self):
        H, d, k = ROUTER_HIDDEN, self.d, self.k
        dev = self._dev()
        W1 = torch.empty((H, d), dtype=torch.float32, device=dev)
        b1 = torch.empty(H, dtype=torch.float32, device=dev)
        W2 = torch.empty((k, H), dtype=torch.float32, device=dev)
        b2 = torch.empty(k, dtype=torch.float32, device=dev)
        self.ctx._sync_stream()
        _check(lib().kmx_router_get_params(self.ctx._p, self._r, _ptr(W1), _ptr(b1), _ptr(W2),
                                           _ptr(b2)), self.ctx._p)
        return W1, b1, W2, b2

    def set_params(self, W1, b1, W2, b2):
        H, d, k = ROUTER_HIDDEN, self.d, self.k
        for t, shape in ((W1, (H, d)), (b1, (H,)), (W2, (k, H)), (b2, (k,))):
            if not t.is_cuda or t.dtype != torch.float32 or tuple(t.shape) != shape \
                    or not t.is_contiguous():
                raise ValueError(f"expected a contiguous float32 CUDA tensor of shape {shape}")
        self.ctx._sync_stream()
        _check(lib().kmx_router_set_params(self.ctx._p, self._r, _ptr(W1), _ptr(b1), _ptr(W2),
                                           _ptr(b2)), self.ctx._p)

    def loss_grad(self, X, labels):
        n, d, ldx = _rows(X)
        _vec(labels, n, torch.int32)
        H, k = ROUTER_HIDDEN, self.k
        dev = self._dev()
        g = (torch.empty((H, d), dtype=torch.float32, device=dev),
             torch.empty(H, dtype=torch.float32, device=dev),
             torch.empty((k, H), dtype=torch.float32, device=dev),
             torch.empty(k, dtype=torch.float32, device=dev))
        loss = ctypes.c_double(0.0)
        self.ctx._sync_stream()
        _check(lib().kmx_router_loss_grad(self.ctx._p, self._r, _ptr(X), n, d, ldx,
                                          _ptr(labels), ctypes.byref(loss), *map(_ptr, g)),
               self.ctx._p)
        return float(loss.value), g

    def train(self, X, labels, epochs: int = 1, batch: int = 8192, lr: float = 1e-3,
              shuffle_seed: int = 1):
        """labels: (n_sets, n) or (n,) int32 CUDA tensor.  Returns per-step losses."""
        n, d, ldx = _rows(X)
        lab = labels if labels.dim() == 2 else labels.view(1, -1)
        if not lab.is_cuda or lab.dtype != torch.int32 or lab.shape[1] != n \
                or not lab.is_contiguous():
            raise ValueError("labels must be a contiguous int32 CUDA tensor of shape (sets, n)")
        sets = lab.shape[0]
        total = n * sets
        steps = epochs * ((total + batch - 1) // batch)
        hist = (ctypes.c_double * max(steps, 1))()
        done = ctypes.c_int64(0)
        self.ctx._sync_stream()
        _check(lib().kmx_router_train(self.ctx._p, self._r, _ptr(X), n, d, ldx, _ptr(lab), sets,
                                      epochs, batch, float(lr),
                                      ctypes.c_uint64(shuffle_seed & (2 ** 64 - 1)), hist,
                                      ctypes.byref(done)), self.ctx._p)
        return [hist[i] for i in range(int(done.value))]

    def propose(self, X):
        n, d, ldx = _rows(X)
        self.ctx._fresh(X)
        cand = torch.empty((n, ROUTER_M), dtype=torch.int32, device=X.device)
        self.ctx._sync_stream()
        _check(lib().kmx_router_propose(self.ctx._p, self._r, _ptr(X), n, d, ldx, _ptr(cand)),
               self.ctx._p)
        return cand


_default = {}


def context(device: int = 0) -> Context:
    """A per-process context for ``device`` (created on first use)."""
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def seed(X, k, w=None, rng_seed=0):
    return context(X.device.index or 0).seed(X, k, w, rng_seed)


def assign(X, C, prec="fp32", want_d=True):
    return context(X.device.index or 0).assign(X, C, prec, want_d)


def update(X, labels, C_prev, w=None, out=None):
    return context(X.device.index or 0).update(X, labels, C_prev, w, out)


def cost(X, C, w=None, prec="fp32"):
    return context(X.device.index or 0).cost(X, C, w, prec)


def lloyd(X, C0, max_iter, w=None, tol=-1.0, prec="bf16", labels=True, inplace=False):
    return context(X.device.index or 0).lloyd(X, C0, max_iter, w, tol, prec, labels, inplace)


class Bico:
    """kmx_bico: the BICO summary (Sec. 2.1, weighted insertion Sec. 2.3.1) of
    at most m features in R^d, kept on the host; the first-level closest
    reference search runs on the context's device."""

    def __init__(self, ctx: Context, d: int, m: int, T0: float):
        self.ctx = ctx
        self.d, self.m = int(d), int(m)
        b = _vp()
        _check(lib().kmx_bico_create(ctx._p, self.d, self.m, float(T0), ctypes.byref(b)), ctx._p)
        self._b = b

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            lib().kmx_bico_destroy(self.ctx._p, self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def insert(self, X, w=None):
        """Insert the rows of X (device, float32) in order, with weights w."""
        n, d, ldx = _rows(X)
        if d != self.d:
            raise ValueError(f"rows of width {d}, summary of width {self.d}")
        _vec(w, n)
        self.ctx._sync_stream()
        _check(lib().kmx_bico_insert(self.ctx._p, self._b, _ptr(X), n, ldx, _ptr(w)), self.ctx._p)

    def stats(self):
        """dict: count, T, rebuilds, gpu_rows, host_scans, pairs."""
        c, r, g, h, pr = (ctypes.c_int64(0) for _ in range(5))
        T = ctypes.c_double(0.0)
        _check(lib().kmx_bico_stats(self.ctx._p, self._b, ctypes.byref(c), ctypes.byref(T),
                                    ctypes.byref(r), ctypes.byref(g), ctypes.byref(h),
                                    ctypes.byref(pr)), self.ctx._p)
        return {"count": int(c.value), "T": float(T.value), "rebuilds": int(r.value),
                "gpu_rows": int(g.value), "host_scans": int(h.value), "pairs": int(pr.value)}

    def features(self):
        """(W, S, Q, ref, level) as numpy arrays, breadth-first order."""
        import numpy as np
        cnt = self.stats()["count"]
        W = np.zeros(cnt, np.float64)
        S = np.zeros((cnt, self.d), np.float64)
        Q = np.zeros(cnt, np.float64)
        R = np.zeros((cnt, self.d), np.float32)
        L = np.zeros(cnt, np.int32)
        _check(lib().kmx_bico_features(self.ctx._p, self._b, W.ctypes.data, S.ctypes.data,
                                       Q.ctypes.data, R.ctypes.data, L.ctypes.data), self.ctx._p)
        return W, S, Q, R, L

    def coreset(self):
        """(P, w) on the device: centroids S / W and weights W."""
        cnt = self.stats()["count"]
        dev = torch.device("cuda", self.ctx.device)
        P = torch.empty((max(cnt, 1), self.d), dtype=torch.float32, device=dev)
        w = torch.empty(max(cnt, 1), dtype=torch.float32, device=dev)
        self.ctx._sync_stream()
        _check(lib().kmx_bico_coreset(self.ctx._p, self._b, _ptr(P), _ptr(w)), self.ctx._p)
        return P[:cnt], w[:cnt]
