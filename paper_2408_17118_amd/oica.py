"""Thin Python binding of liboica (include/oica.h) over ctypes.

Argument marshalling only: every step of the path runs in the HIP kernels of
liboica.so.  PyTorch provides device memory and the stream.  If the shared
library is missing, every call raises; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liboica.so")
_lib = None

OICA_F64, OICA_F32, OICA_BF16 = 0, 1, 2
ROW_NOTCONV, ROW_CONV, ROW_PRUNED, ROW_DEGENERATE = 0, 1, 2, 3
MAX_N = 128

ERRORS = {
    0: "OICA_OK", -1: "OICA_E_ARG", -2: "OICA_E_SHAPE", -3: "OICA_E_RANK",
    -4: "OICA_E_NONFINITE", -5: "OICA_E_DEVICE", -6: "OICA_E_NOMEM", -7: "OICA_E_UNSUPPORTED",
    -8: "OICA_E_NOCONV",
}
OPT_COOP_GIVE_UP, OPT_JACOBI_MAX_SWEEPS, OPT_COOP_FALLBACKS, OPT_COOP_LAUNCH_API = 1, 2, 3, 4


class OicaError(RuntimeError):
    def __init__(self, code: int, detail: str):
        super().__init__(f"{ERRORS.get(code, code)}: {detail}")
        self.code = code
        self.detail = detail


class FpParams(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("tol", C.c_double), ("precision", C.c_int),
                ("tol_bf16", C.c_double), ("refine_iters", C.c_int), ("traj_iters", C.c_int),
                ("check_every", C.c_int), ("profile", C.c_int), ("refine_groups", C.c_int),
                ("pruner", C.c_void_p), ("prune_pass", C.c_int), ("guard_top", C.c_int),
                ("guard_min", C.c_int), ("bf16_row_terms", C.c_int),
                ("bf16_switch_step", C.c_double)]


class FpStats(C.Structure):
    _fields_ = [("thread_iters", C.c_int64), ("passes", C.c_int),
                ("refine_thread_iters", C.c_int64), ("ms", C.c_double),
                ("update_ms", C.c_double), ("update_launches", C.c_int),
                ("pruned", C.c_int), ("guard_tripped", C.c_int)]


class WhitenProblem(C.Structure):
    _fields_ = [("N", C.c_int), ("T", C.c_int64), ("X_raw", C.c_void_p), ("raw_t", C.c_int),
                ("ld_raw", C.c_int64), ("Xw", C.c_void_p), ("Xw_f32", C.c_void_p), ("V", C.c_void_p),
                ("mean", C.c_void_p), ("eigval", C.c_void_p), ("status", C.c_int)]


class Problem(C.Structure):
    _fields_ = [("N", C.c_int), ("T", C.c_int64), ("K", C.c_int), ("Xw", C.c_void_p),
                ("Xw_f32", C.c_void_p), ("W0", C.c_void_p), ("W_out", C.c_void_p),
                ("kurt", C.c_void_p), ("iters", C.c_void_p), ("status", C.c_void_p)]


class BatchParams(C.Structure):
    _fields_ = [("autotune", C.c_int), ("cache_path", C.c_char_p), ("force_wk", C.c_int),
                ("force_grid", C.c_int)]


class BatchStats(C.Structure):
    _fields_ = [("thread_iters", C.c_int64), ("refine_thread_iters", C.c_int64),
                ("passes", C.c_int), ("ms", C.c_double), ("update_ms", C.c_double),
                ("update_launches", C.c_int), ("grid", C.c_int), ("wk32", C.c_int),
                ("wk64", C.c_int), ("tuned", C.c_int), ("update_flops", C.c_double)]


class UniqueProblem(C.Structure):
    _fields_ = [("N", C.c_int), ("T", C.c_int64), ("K", C.c_int), ("W", C.c_void_p),
                ("kurt", C.c_void_p), ("status", C.c_void_p), ("cap", C.c_int),
                ("U", C.c_void_p), ("kurt_u", C.c_void_p), ("ups_u", C.c_void_p),
                ("rep_thread", C.c_void_p), ("cluster_size", C.c_void_p),
                ("row_cluster", C.c_void_p), ("n_unique", C.c_int), ("n_accepted", C.c_int)]


class UniqueParams(C.Structure):
    _fields_ = [("tau", C.c_double), ("gaussianity_test", C.c_int), ("n_top", C.c_int)]


class DeflationStep(C.Structure):
    _fields_ = [("dim", C.c_int), ("rep", C.c_int), ("accepted", C.c_int), ("passes", C.c_int),
                ("thread_iters", C.c_int64), ("refine_thread_iters", C.c_int64),
                ("alpha", C.c_double), ("upsilon", C.c_double), ("threshold", C.c_double)]


_P = C.c_void_p
_SIGS = {
    "oica_version": (C.c_int, []),
    "oica_create": (C.c_int, [C.POINTER(_P), C.c_int, _P]),
    "oica_destroy": (None, [_P]),
    "oica_status_string": (C.c_char_p, [C.c_int]),
    "oica_last_error": (C.c_char_p, [_P]),
    "oica_set_stream": (C.c_int, [_P, _P]),
    "oica_whiten": (C.c_int, [_P, C.c_int, C.c_int64, _P, C.c_int, C.c_int64, _P, C.c_int, _P, _P,
                              _P, _P]),
    "oica_whiten_batched": (C.c_int, [_P, C.c_int, C.POINTER(WhitenProblem), C.c_int]),
    "oica_fixed_point": (C.c_int, [_P, C.c_int, C.c_int64, _P, C.c_int, _P, C.c_int, _P,
                                   C.POINTER(FpParams), _P, _P, _P, _P, _P, C.POINTER(FpStats)]),
    "oica_update": (C.c_int, [_P, C.c_int, C.c_int64, _P, C.c_int, C.c_int, _P, _P, _P]),
    "oica_kurtosis": (C.c_int, [_P, C.c_int, C.c_int64, _P, C.c_int, _P, _P]),
    "oica_kurtosis_noalloc": (C.c_int, [_P, C.c_int, C.c_int64, _P, C.c_int, _P, _P]),
    "oica_fixed_point_batched": (C.c_int, [_P, C.c_int, C.POINTER(Problem), C.c_int,
                                           C.POINTER(FpParams), C.POINTER(BatchParams),
                                           C.POINTER(BatchStats)]),
    "oica_pruner_create": (C.c_int, [_P, _P, _P, _P, C.POINTER(_P)]),
    "oica_pruner_destroy": (None, [_P]),
    "oica_pruner_get_weights": (C.c_int, [_P, _P, _P]),
    "oica_pruner_set_threshold": (C.c_int, [_P, C.c_float]),
    "oica_pruner_predict": (C.c_int, [_P, _P, _P, C.c_int64, _P]),
    "oica_pruner_grad": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.c_float, _P,
                                   C.POINTER(C.c_double)]),
    "oica_pruner_train_step": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.c_float, C.c_float,
                                         C.POINTER(C.c_double)]),
    "oica_pruner_train": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.c_int, C.c_int, C.c_float,
                                    C.c_float, C.c_uint64, _P]),
    "oica_unique": (C.c_int, [_P, C.c_int, C.c_int64, C.c_int, _P, _P, _P, C.POINTER(UniqueParams),
                              C.c_int, _P, _P, _P, _P, _P, _P, C.POINTER(C.c_int),
                              C.POINTER(C.c_int)]),
    "oica_set_option": (C.c_int, [C.c_int, C.c_int]),
    "oica_get_option": (C.c_int, [C.c_int, C.POINTER(C.c_int)]),
    "oica_deflation": (C.c_int, [_P, C.c_int, C.c_int64, _P, C.c_int, _P, C.POINTER(FpParams),
                                 C.c_double, C.c_int, _P, C.POINTER(C.c_int),
                                 C.POINTER(DeflationStep)]),
    "oica_ordering_original": (C.c_int, [_P, C.c_int, C.c_int64, _P, C.c_int, _P,
                                         C.POINTER(FpParams), C.c_double, C.c_int, _P,
                                         C.POINTER(C.c_int), C.POINTER(DeflationStep)]),
    "oica_unique_batched": (C.c_int, [_P, C.c_int, C.POINTER(UniqueProblem),
                                      C.POINTER(UniqueParams)]),
}


def lib_path() -> str:
    return _LIB_PATH


def load():
    """Load liboica.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise OicaError(-5, f"{_LIB_PATH} not built; run python -m paper_2408_17118_amd.build")
        lib = C.CDLL(_LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def exported_symbols() -> list[str]:
    return list(_SIGS)


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _ld(X):
    """Row stride in elements of a checked row-strided matrix (a single row's
    stride is meaningless, so its length stands in)."""
    return X.stride(0) if X.shape[0] > 1 else X.shape[1]


def _dev(t, name, dtype=None, shape=None, row_strided=False):
    """Check a device argument before its pointer crosses the C ABI, which
    cannot see dtypes or sizes: dtype (one or a tuple) and shape (None entries
    match any size) as the call documents.  row_strided: a 2-D matrix whose
    rows are contiguous but may lie further apart than their length (the call
    takes the row stride)."""
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if row_strided and t.dim() == 2:
        if (t.shape[1] > 1 and t.stride(1) != 1) or (t.shape[0] > 1 and t.stride(0) < t.shape[1]):
            raise ValueError(f"{name} must have contiguous rows (stride(1) == 1, "
                             f"stride(0) >= {t.shape[1]}), not strides {tuple(t.stride())}")
    elif not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None:
        ok = dtype if isinstance(dtype, tuple) else (dtype,)
        if t.dtype not in ok:
            raise TypeError(f"{name} must have dtype {' or '.join(str(d) for d in ok)}, not {t.dtype}")
    if shape is not None:
        if t.dim() != len(shape) or any(w is not None and w != v for w, v in zip(shape, t.shape)):
            raise ValueError(f"{name} must have shape {tuple(shape)}, not {tuple(t.shape)}")
    return t


_DT = {torch.float64: OICA_F64, torch.float32: OICA_F32, torch.bfloat16: OICA_BF16}


class Context:
    """An oica_ctx bound to one device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        self.lib = load()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        rc = self.lib.oica_create(C.byref(h), device, C.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise OicaError(rc, "oica_create failed")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            self.lib.oica_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise OicaError(rc, (self.lib.oica_last_error(self.h) or b"").decode())

    def _tdev(self):
        return torch.device("cuda", self.device)

    # ---- a1-a3 ------------------------------------------------------------
    def whiten(self, X: torch.Tensor, out_dtype=torch.float32, want_f32=True):
        """X: N x T raw data (float64 or float32, device; rows contiguous, and
        may be a column window of a longer recording).  Returns
        (Xw, Xw_f32, V, mean, eigval); Xw_f32 is Xw itself for FP32 output."""
        _dev(X, "X", (torch.float64, torch.float32), (None, None), row_strided=True)
        N, T = X.shape
        dev = self._tdev()
        Xw = torch.empty((N, T), dtype=out_dtype, device=dev)
        Xw32 = None
        if out_dtype == torch.bfloat16 and want_f32:
            Xw32 = torch.empty((N, T), dtype=torch.float32, device=dev)
        V = torch.empty((N, N), dtype=torch.float64, device=dev)
        mean = torch.empty(N, dtype=torch.float64, device=dev)
        eig = torch.empty(N, dtype=torch.float64, device=dev)
        rc = self.lib.oica_whiten(self.h, N, T, _ptr(X), _DT[X.dtype], _ld(X), _ptr(Xw),
                                  _DT[out_dtype], _ptr(Xw32), _ptr(V), _ptr(mean), _ptr(eig))
        self._check(rc)
        return Xw, (Xw if out_dtype == torch.float32 else Xw32), V, mean, eig

    def whiten_batched(self, Xs, out_dtype=torch.float32, want_f32=True, return_status=False):
        """Xs: list of N_d x T_d raw device tensors.  Returns a list of
        (Xw, Xw_f32, V, mean, eigval) per dataset, as whiten() does; with
        return_status, also the per-dataset codes, and data errors (rank,
        non-finite) do not raise."""
        D = len(Xs)
        arr = (WhitenProblem * D)()
        dev = self._tdev()
        outs = []
        for d, X in enumerate(Xs):
            _dev(X, "X", (torch.float64, torch.float32), (None, None), row_strided=True)
            N, T = X.shape
            Xw = torch.empty((N, T), dtype=out_dtype, device=dev)
            Xw32 = None
            if out_dtype == torch.bfloat16 and want_f32:
                Xw32 = torch.empty((N, T), dtype=torch.float32, device=dev)
            V = torch.empty((N, N), dtype=torch.float64, device=dev)
            mean = torch.empty(N, dtype=torch.float64, device=dev)
            eig = torch.empty(N, dtype=torch.float64, device=dev)
            arr[d] = WhitenProblem(N, T, _ptr(X), _DT[X.dtype], _ld(X), _ptr(Xw), _ptr(Xw32),
                                   _ptr(V), _ptr(mean), _ptr(eig), 0)
            outs.append((Xw, (Xw if out_dtype == torch.float32 else Xw32), V, mean, eig))
        rc = self.lib.oica_whiten_batched(self.h, D, arr, _DT[out_dtype])
        if return_status and rc in (-3, -4, -8):
            return outs, [arr[d].status for d in range(D)]
        self._check(rc)
        return (outs, [arr[d].status for d in range(D)]) if return_status else outs

    # ---- a4-a11, a14 ----------------------------------------------------------
    def fixed_point(self, Xw, W0, Xw_f32=None, max_iter=1000, tol=1e-6, precision="f32",
                    tol_bf16=1e-3, refine_iters=5, traj_iters=0, check_every=4, profile=False,
                    refine_groups=True, pruner=None, prune_pass=8, guard_top=0, guard_min=4,
                    bf16_row_terms=0, bf16_switch_step=0.0):
        _dev(Xw, "Xw", torch.bfloat16 if precision == "bf16" else torch.float32, (None, None))
        N, T = Xw.shape
        _dev(W0, "W0", torch.float32, (None, N))
        K = W0.shape[0]
        if Xw_f32 is None:
            Xw_f32 = Xw
        _dev(Xw_f32, "Xw_f32", torch.float32, (N, T))
        dev = self._tdev()
        W = torch.empty((K, N), dtype=torch.float32, device=dev)
        kurt = torch.empty(K, dtype=torch.float64, device=dev)
        iters = torch.empty(K, dtype=torch.int32, device=dev)
        status = torch.empty(K, dtype=torch.uint8, device=dev)
        traj = torch.empty((K, traj_iters, 2), dtype=torch.float32, device=dev) if traj_iters else None
        p = FpParams(max_iter, tol, OICA_BF16 if precision == "bf16" else OICA_F32, tol_bf16,
                     refine_iters, traj_iters, check_every, 1 if profile else 0,
                     1 if refine_groups else 0, pruner.h if pruner is not None else None,
                     prune_pass, guard_top, guard_min, bf16_row_terms, bf16_switch_step)
        st = FpStats()
        rc = self.lib.oica_fixed_point(self.h, N, T, _ptr(Xw), _DT[Xw.dtype], _ptr(Xw_f32), K,
                                       _ptr(W0), C.byref(p), _ptr(W), _ptr(kurt), _ptr(iters),
                                       _ptr(status), _ptr(traj), C.byref(st))
        self._check(rc)
        return {"W": W, "kurt": kurt, "iters": iters, "status": status, "traj": traj,
                "thread_iters": int(st.thread_iters), "passes": int(st.passes),
                "refine_thread_iters": int(st.refine_thread_iters), "ms": float(st.ms),
                "update_ms": float(st.update_ms), "update_launches": int(st.update_launches),
                "pruned": int(st.pruned), "guard_tripped": int(st.guard_tripped)}

    def fixed_point_batched(self, problems, max_iter=1000, tol=1e-6, precision="f32",
                            tol_bf16=1e-3, refine_iters=5, check_every=4, profile=False,
                            autotune=True, cache_path=None, force_wk=0, force_grid=0,
                            refine_groups=True, bf16_row_terms=0):
        """problems: list of dicts with device tensors Xw (N x T), W0 (K x N float32) and,
        for BF16 data, Xw_f32.  Returns (list of per-problem outputs, stats dict)."""
        D = len(problems)
        arr = (Problem * D)()
        outs = []
        dev = self._tdev()
        for d, q in enumerate(problems):
            Xw = _dev(q["Xw"], f"problem {d} Xw",
                      torch.bfloat16 if precision == "bf16" else torch.float32, (None, None))
            N, T = Xw.shape
            X32 = _dev(q.get("Xw_f32", Xw), f"problem {d} Xw_f32", torch.float32, (N, T))
            W0 = _dev(q["W0"], f"problem {d} W0", torch.float32, (None, N))
            K = W0.shape[0]
            o = {"W": torch.empty((K, N), dtype=torch.float32, device=dev),
                 "kurt": torch.empty(K, dtype=torch.float64, device=dev),
                 "iters": torch.empty(K, dtype=torch.int32, device=dev),
                 "status": torch.empty(K, dtype=torch.uint8, device=dev)}
            arr[d] = Problem(N, T, K, Xw.data_ptr(), X32.data_ptr(), W0.data_ptr(),
                             o["W"].data_ptr(), o["kurt"].data_ptr(), o["iters"].data_ptr(),
                             o["status"].data_ptr())
            o["_keep"] = (Xw, X32, W0)
            outs.append(o)
        xw_t = OICA_BF16 if precision == "bf16" else OICA_F32
        p = FpParams(max_iter, tol, xw_t, tol_bf16, refine_iters, 0, check_every,
                     1 if profile else 0, 1 if refine_groups else 0, None, 0, 0, 0,
                     bf16_row_terms)
        bp = BatchParams(1 if autotune else 0, cache_path.encode() if cache_path else None,
                         force_wk, force_grid)
        st = BatchStats()
        rc = self.lib.oica_fixed_point_batched(self.h, D, arr, xw_t, C.byref(p), C.byref(bp),
                                               C.byref(st))
        self._check(rc)
        for o in outs:
            o.pop("_keep")
        stats = {k: getattr(st, k) for k, _ in BatchStats._fields_}
        return outs, stats

    def update(self, Xw, B):
        _dev(Xw, "Xw", (torch.float32, torch.bfloat16), (None, None))
        N, T = Xw.shape
        _dev(B, "B", torch.float32, (None, N))
        K = B.shape[0]
        G = torch.empty((K, N), dtype=torch.float64, device=self._tdev())
        s4 = torch.empty(K, dtype=torch.float64, device=self._tdev())
        rc = self.lib.oica_update(self.h, N, T, _ptr(Xw), _DT[Xw.dtype], K, _ptr(B), _ptr(G), _ptr(s4))
        self._check(rc)
        return G, s4

    def kurtosis(self, Xw_f32, W):
        _dev(Xw_f32, "Xw_f32", torch.float32, (None, None))
        N, T = Xw_f32.shape
        _dev(W, "W", torch.float32, (None, N))
        K = W.shape[0]
        kurt = torch.empty(K, dtype=torch.float64, device=self._tdev())
        rc = self.lib.oica_kurtosis(self.h, N, T, _ptr(Xw_f32), K, _ptr(W), _ptr(kurt))
        self._check(rc)
        return kurt

    def kurtosis_noalloc(self, Xw_f32, W, kurt):
        """oica_kurtosis_noalloc: the library allocates nothing; the caller passes
        the output ``kurt`` (K float64 on the device)."""
        _dev(Xw_f32, "Xw_f32", torch.float32, (None, None))
        N, T = Xw_f32.shape
        _dev(W, "W", torch.float32, (None, N))
        K = W.shape[0]
        _dev(kurt, "kurt", torch.float64, (K,))
        rc = self.lib.oica_kurtosis_noalloc(self.h, N, T, _ptr(Xw_f32), K, _ptr(W), _ptr(kurt))
        self._check(rc)
        return kurt

    # ---- deflation driver (Algorithm 2's outer loop) ------------------------------
    def deflation(self, Xw, W0_blocks, max_iter=1000, tol=1e-6, precision="f32", tol_bf16=1e-3,
                  refine_iters=5, tau=1e-3, check_every=4, gaussianity_test=True):
        """Xw: N x T float32 whitened data; W0_blocks: the start rows of every
        step, step i's block L x (N - i + 1) float32 (a list of N tensors, or
        one flat device tensor holding them one after the other).  Returns
        (W: n_found x N float64 device tensor, list of per-step dicts)."""
        _dev(Xw, "Xw", torch.float32, (None, None))
        N, T = Xw.shape
        if isinstance(W0_blocks, (list, tuple)):
            if len(W0_blocks) != N:
                raise ValueError(f"W0_blocks must hold {N} blocks, not {len(W0_blocks)}")
            L = W0_blocks[0].shape[0]
            for i, b in enumerate(W0_blocks):
                _dev(b, f"W0_blocks[{i}]", torch.float32, (L, N - i))
            flat = torch.cat([b.reshape(-1) for b in W0_blocks])
        else:
            flat = _dev(W0_blocks, "W0_blocks", torch.float32, (None,))
            L = flat.numel() // (N * (N + 1) // 2)
            if L * (N * (N + 1) // 2) != flat.numel() or L < 1:
                raise ValueError("flat W0_blocks must hold L N (N + 1) / 2 values")
        W = torch.zeros((N, N), dtype=torch.float64, device=self._tdev())
        p = FpParams(max_iter, tol, OICA_BF16 if precision == "bf16" else OICA_F32, tol_bf16,
                     refine_iters, 0, check_every, 0, 1, None, 0, 0, 0)
        steps = (DeflationStep * N)()
        n_found = C.c_int(0)
        rc = self.lib.oica_deflation(self.h, N, T, _ptr(Xw), L, _ptr(flat), C.byref(p), float(tau),
                                     1 if gaussianity_test else 0, _ptr(W), C.byref(n_found), steps)
        self._check(rc)
        taken = []
        for i in range(N):
            st = steps[i]
            if st.dim == 0:
                break
            taken.append({k: getattr(st, k) for k, _ in DeflationStep._fields_})
            if not st.accepted:
                break
        return W[: n_found.value], taken

    def ordering_original(self, Xw, W0_blocks, max_iter=1000, tol=1e-6, tau=1e-3,
                          check_every=4, gaussianity_test=True):
        """Algorithm 1 as a batched variant (oica_ordering_original).  Xw: N x T
        float32; W0_blocks: N blocks of L x N float32 start rows (a list, or one
        flat tensor).  Returns (W: n_found x N float64, per-step dicts)."""
        _dev(Xw, "Xw", torch.float32, (None, None))
        N, T = Xw.shape
        if isinstance(W0_blocks, (list, tuple)):
            if len(W0_blocks) != N:
                raise ValueError(f"W0_blocks must hold {N} blocks, not {len(W0_blocks)}")
            L = W0_blocks[0].shape[0]
            for i, b in enumerate(W0_blocks):
                _dev(b, f"W0_blocks[{i}]", torch.float32, (L, N))
            flat = torch.cat([b.reshape(-1) for b in W0_blocks])
        else:
            flat = _dev(W0_blocks, "W0_blocks", torch.float32, (None,))
            L = flat.numel() // (N * N)
            if L * N * N != flat.numel() or L < 1:
                raise ValueError("flat W0_blocks must hold L N N values")
        W = torch.zeros((N, N), dtype=torch.float64, device=self._tdev())
        p = FpParams(max_iter, tol, OICA_F32, 1e-5, 0, 0, check_every, 0, 1, None, 0, 0, 0)
        steps = (DeflationStep * N)()
        n_found = C.c_int(0)
        rc = self.lib.oica_ordering_original(self.h, N, T, _ptr(Xw), L, _ptr(flat), C.byref(p),
                                             float(tau), 1 if gaussianity_test else 0, _ptr(W),
                                             C.byref(n_found), steps)
        self._check(rc)
        taken = []
        for i in range(N):
            st = steps[i]
            if st.dim == 0:
                break
            taken.append({k: getattr(st, k) for k, _ in DeflationStep._fields_})
            if not st.accepted:
                break
        return W[: n_found.value], taken

    # ---- a12-a13 ----------------------------------------------------------------
    def unique(self, W, kurt, status, T, tau=1e-3, gaussianity_test=True, n_top=0, cap=None,
               row_cluster=False):
        _dev(W, "W", torch.float32, (None, None))
        K, N = W.shape
        _dev(kurt, "kurt", torch.float64, (K,))
        _dev(status, "status", torch.uint8, (K,))
        cap = K if cap is None else cap
        dev = self._tdev()
        U = torch.empty((max(cap, 1), N), dtype=torch.float64, device=dev)
        ku = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
        uu = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
        rep = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        size = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        rc_rows = torch.empty(K, dtype=torch.int32, device=dev) if row_cluster else None
        nu, na = C.c_int(), C.c_int()
        p = UniqueParams(tau, 1 if gaussianity_test else 0, n_top)
        rc = self.lib.oica_unique(self.h, N, T, K, _ptr(W), _ptr(kurt), _ptr(status), C.byref(p), cap,
                                  _ptr(U), _ptr(ku), _ptr(uu), _ptr(rep), _ptr(size), _ptr(rc_rows),
                                  C.byref(nu), C.byref(na))
        self._check(rc)
        n = nu.value
        out = {"U": U[:n], "alpha": ku[:n], "upsilon": uu[:n], "rep": rep[:n], "size": size[:n],
               "n_unique": n, "n_accepted": na.value}
        if row_cluster:
            out["row_cluster"] = rc_rows
        return out

    def unique_batched(self, items, tau=1e-3, gaussianity_test=True, n_top=0, row_cluster=False):
        """items: list of (W, kurt, status, T).  Returns a list of dicts as unique() does."""
        D = len(items)
        arr = (UniqueProblem * D)()
        dev = self._tdev()
        outs = []
        for d, (W, kurt, status, T) in enumerate(items):
            _dev(W, f"item {d} W", torch.float32, (None, None))
            K, N = W.shape
            _dev(kurt, f"item {d} kurt", torch.float64, (K,))
            _dev(status, f"item {d} status", torch.uint8, (K,))
            o = {"U": torch.empty((K, N), dtype=torch.float64, device=dev),
                 "alpha": torch.empty(K, dtype=torch.float64, device=dev),
                 "upsilon": torch.empty(K, dtype=torch.float64, device=dev),
                 "rep": torch.empty(K, dtype=torch.int32, device=dev),
                 "size": torch.empty(K, dtype=torch.int32, device=dev)}
            if row_cluster:
                o["row_cluster"] = torch.empty(K, dtype=torch.int32, device=dev)
            arr[d] = UniqueProblem(N, T, K, _ptr(W), _ptr(kurt), _ptr(status), K, _ptr(o["U"]),
                                   _ptr(o["alpha"]), _ptr(o["upsilon"]), _ptr(o["rep"]),
                                   _ptr(o["size"]), _ptr(o.get("row_cluster")), 0, 0)
            outs.append(o)
        p = UniqueParams(tau, 1 if gaussianity_test else 0, n_top)
        rc = self.lib.oica_unique_batched(self.h, D, arr, C.byref(p))
        self._check(rc)
        for d, o in enumerate(outs):
            n = arr[d].n_unique
            for k in ("U", "alpha", "upsilon", "rep", "size"):
                o[k] = o[k][:n]
            o["n_unique"] = n
            o["n_accepted"] = arr[d].n_accepted
        return outs


class Pruner:
    """The learned pruner (weights on the context's device)."""

    N_PARAMS = 5313

    def __init__(self, ctx: Context, init_w, feat_mean, feat_std):
        import numpy as np
        self.ctx = ctx
        w = np.ascontiguousarray(init_w, dtype=np.float32)
        m = np.ascontiguousarray(feat_mean, dtype=np.float32)
        sd = np.ascontiguousarray(feat_std, dtype=np.float32)
        if w.size != self.N_PARAMS or m.size != 16 or sd.size != 16:
            raise ValueError("pruner needs 5313 weights and 16 feature means / stds")
        h = C.c_void_p()
        rc = ctx.lib.oica_pruner_create(ctx.h, w.ctypes.data, m.ctypes.data, sd.ctypes.data,
                                        C.byref(h))
        ctx._check(rc)
        self.h = h
        self.feat_mean, self.feat_std = m, sd

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.oica_pruner_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def weights(self):
        import numpy as np
        out = np.empty(self.N_PARAMS, dtype=np.float32)
        self.ctx._check(self.ctx.lib.oica_pruner_get_weights(self.ctx.h, self.h, out.ctypes.data))
        return out

    def set_threshold(self, theta: float):
        self.ctx._check(self.ctx.lib.oica_pruner_set_threshold(self.h, float(theta)))
        self.theta = float(theta)

    def predict(self, traj):
        _dev(traj, "traj", torch.float32, (None, 8, 2))
        R = traj.shape[0]
        prob = torch.empty(R, dtype=torch.float32, device=traj.device)
        self.ctx._check(self.ctx.lib.oica_pruner_predict(self.ctx.h, self.h, _ptr(traj), R,
                                                         _ptr(prob)))
        return prob

    def grad(self, traj, labels, w_pos):
        _dev(traj, "traj", torch.float32, (None, 8, 2))
        R = traj.shape[0]
        _dev(labels, "labels", torch.uint8, (R,))
        g = torch.empty(self.N_PARAMS, dtype=torch.float32, device=traj.device)
        loss = C.c_double()
        self.ctx._check(self.ctx.lib.oica_pruner_grad(self.ctx.h, self.h, _ptr(traj), _ptr(labels),
                                                      R, float(w_pos), _ptr(g), C.byref(loss)))
        return g, loss.value

    def train_step(self, traj, labels, w_pos, lr=1e-3):
        _dev(traj, "traj", torch.float32, (None, 8, 2))
        R = traj.shape[0]
        _dev(labels, "labels", torch.uint8, (R,))
        loss = C.c_double()
        self.ctx._check(self.ctx.lib.oica_pruner_train_step(self.ctx.h, self.h, _ptr(traj),
                                                            _ptr(labels), R, float(w_pos),
                                                            float(lr), C.byref(loss)))
        return loss.value

    def train(self, traj, labels, epochs=4, batch=65536, lr=2e-3, seed=0, w_pos=0.0):
        """Whole training run in the library (shuffled epochs of batch-row Adam
        steps); w_pos 0 weighs positives by n_neg / n_pos.  Returns the mean
        loss of each epoch."""
        import numpy as np
        _dev(traj, "traj", torch.float32, (None, 8, 2))
        R = traj.shape[0]
        _dev(labels, "labels", torch.uint8, (R,))
        out = np.zeros(int(epochs), dtype=np.float64)
        self.ctx._check(self.ctx.lib.oica_pruner_train(self.ctx.h, self.h, _ptr(traj), _ptr(labels),
                                                       R, int(epochs), int(batch), float(w_pos),
                                                       float(lr), int(seed) & (2**64 - 1),
                                                       out.ctypes.data))
        return [float(x) for x in out]


def set_option(option: int, value: int) -> None:
    """oica_set_option: process-wide switches for tests of failure handling."""
    rc = load().oica_set_option(int(option), int(value))
    if rc:
        raise OicaError(rc, f"option {option} = {value}")


def get_option(option: int) -> int:
    v = C.c_int(0)
    rc = load().oica_get_option(int(option), C.byref(v))
    if rc:
        raise OicaError(rc, f"option {option}")
    return v.value


def ordering_ica(ctx: Context, X: torch.Tensor, W0: torch.Tensor, tol=1e-6, max_iter=1000,
                 tau=1e-3, gaussianity_test=True, precision="f32", tol_bf16=1e-3, refine_iters=5,
                 profile=False, refine_groups=True, pruner=None, traj_iters=0, bf16_row_terms=0,
                 bf16_switch_step=0.0):
    """Whole hot path on device-resident raw data: whiten -> fixed point -> unique."""
    xw_dtype = torch.bfloat16 if precision == "bf16" else torch.float32
    Xw, Xw32, V, mean, eig = ctx.whiten(X, out_dtype=xw_dtype)
    fp = ctx.fixed_point(Xw, W0, Xw_f32=Xw32, max_iter=max_iter, tol=tol, precision=precision,
                         tol_bf16=tol_bf16, refine_iters=refine_iters, profile=profile,
                         refine_groups=refine_groups, pruner=pruner, traj_iters=traj_iters,
                         bf16_row_terms=bf16_row_terms, bf16_switch_step=bf16_switch_step)
    res = ctx.unique(fp["W"], fp["kurt"], fp["status"], X.shape[1], tau=tau,
                     gaussianity_test=gaussianity_test)
    res.update(fp=fp, V=V, mean=mean, eig=eig, Xw=Xw, Xw_f32=Xw32)
    return res


def ordering_ica_deflation(ctx: Context, X: torch.Tensor, W0_blocks, tol=1e-6, max_iter=1000,
                           tau=1e-3, precision="f32", tol_bf16=1e-3, refine_iters=5):
    """The paper's full method on device-resident raw data: whiten, then the
    deflation driver (one component per step).  Returns a dict with the
    components in whitened space (W), in raw-data space (W V, unit rows), the
    per-step records and the whitening outputs."""
    Xw, Xw32, V, mean, eig = ctx.whiten(X, out_dtype=torch.float32)
    W, steps = ctx.deflation(Xw32, W0_blocks, max_iter=max_iter, tol=tol, precision=precision,
                             tol_bf16=tol_bf16, refine_iters=refine_iters, tau=tau)
    Wr = W @ V
    Wr = Wr / torch.linalg.norm(Wr, dim=1, keepdim=True)
    return {"W": W, "W_raw": Wr, "steps": steps, "V": V, "mean": mean, "eig": eig, "Xw": Xw32}


def ordering_ica_batched(ctx: Context, Xs, W0s, tol=1e-6, max_iter=1000, tau=1e-3,
                         gaussianity_test=True, precision="f32", tol_bf16=1e-3, refine_iters=5,
                         profile=False, autotune=True, cache_path=None, refine_groups=True):
    """Whole hot path for many device-resident raw datasets: whiten each, one
    batched fixed point over all of them, unique set of each.  Returns (list of
    per-dataset results as from ordering_ica, batched stats)."""
    xw_dtype = torch.bfloat16 if precision == "bf16" else torch.float32
    probs, wh = [], []
    for (Xw, Xw32, V, mean, eig), W0 in zip(ctx.whiten_batched(Xs, out_dtype=xw_dtype), W0s):
        probs.append({"Xw": Xw, "Xw_f32": Xw32, "W0": W0})
        wh.append((V, mean, eig))
    outs, st = ctx.fixed_point_batched(probs, max_iter=max_iter, tol=tol, precision=precision,
                                       tol_bf16=tol_bf16, refine_iters=refine_iters,
                                       profile=profile, autotune=autotune, cache_path=cache_path,
                                       refine_groups=refine_groups)
    res = ctx.unique_batched([(o["W"], o["kurt"], o["status"], X.shape[1])
                              for X, o in zip(Xs, outs)], tau=tau,
                             gaussianity_test=gaussianity_test)
    for r, o, (V, mean, eig) in zip(res, outs, wh):
        r.update(fp=o, V=V, mean=mean, eig=eig)
    return res, st
