"""Python binding of libasi (include/asi.h): argument marshalling only.

Every numeric step runs in the library's HIP kernels; PyTorch supplies device
memory (the workspace and the input/output tensors) and the stream. The
binding loads the in-tree ``libasi.so`` and fails loudly when it is missing;
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libasi.so")

STATUS = {0: "ASI_OK", 1: "ASI_E_ARG", 2: "ASI_E_PATTERN", 3: "ASI_E_SINGULAR_D",
          4: "ASI_E_NONFINITE", 5: "ASI_E_STATE", 6: "ASI_E_WORKSPACE", 7: "ASI_E_HIP",
          8: "ASI_E_UNSUPPORTED", 9: "ASI_E_TIMEOUT"}
SWEEP = {"auto": 0, "levels": 1, "dataflow": 2}
PRECISION = {"fp64": 0, "mixed": 1}

# every symbol the header declares
EXPORTS = ["asi_create", "asi_destroy", "asi_set_stream", "asi_last_error", "asi_analyze",
           "asi_set_workspace", "asi_get_info", "asi_get_pattern", "asi_selinv", "asi_ninv",
           "asi_mix", "asi_spai", "asi_lowrank", "asi_diag", "asi_sync", "asi_profile",
           "asi_profile_read", "asi_set_sweep", "asi_mlp_features", "asi_mlp_pack", "asi_mlp_forward",
           "asi_mlp_backward", "asi_mlp_loss", "asi_mlp_adam", "asi_mlp_apply", "asi_diag_err1", "asi_mlp_correct", "asi_load_factor", "asi_selinv_ninv", "asi_trace", "asi_ninv_full", "asi_mix_full",
           "asi_spmv", "asi_ldl_solve", "asi_pcg", "asi_sqmr", "asi_za_diag", "asi_check_matrix",
           "asi_eigs_work_bytes", "asi_eigs_error", "asi_dense_symeig", "asi_block_solve_work_bytes",
           "asi_pcg_block", "asi_sqmr_block", "asi_mlp_correct_mix", "asi_ildl_numeric",
           "asi_sweep_plan", "asi_unpermute", "asi_unpermute_noalloc", "asi_ildl_threshold_work_bytes",
           "asi_ildl_threshold", "asi_ildl_threshold_extract", "asi_set_sentinel"]
MLP_FEATURES = 16
MLP_PARAMS = 5313
MLP_PACKED_BYTES = 12944
SWEEP_VARIANTS = ["small", "split", "group128", "group256", "group512", "big256", "big1024"]
KERNEL_CLASSES = {"dinv": 0, "selinv": 1, "selinv_big": 2, "ninv": 3, "mix": 4, "spai": 5,
                  "lowrank": 6, "gather_l": 7, "selinv_flow": 8, "mlp_features": 9, "mlp_forward": 10,
                  "mlp_train": 11, "diag": 12, "ildl": 13}


class AsiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_blocks", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("max_cols", ctypes.c_int32), ("nnz_L", ctypes.c_int64), ("nnz_S", ctypes.c_int64),
                ("gather_pairs", ctypes.c_int64), ("gather_hits", ctypes.c_int64),
                ("workspace_min", ctypes.c_size_t), ("workspace_default", ctypes.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library():
    """Load the in-tree libasi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first (__graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "asi_create": [ctypes.POINTER(P), ctypes.c_int, P],
        "asi_destroy": [P],
        "asi_set_stream": [P, P],
        "asi_analyze": [P, i32, P, P, P, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_size_t)],
        "asi_set_workspace": [P, P, ctypes.c_size_t],
        "asi_get_info": [P, ctypes.POINTER(Info)],
        "asi_get_pattern": [P, P, P, P],
        "asi_load_factor": [P, P, P, P],
        "asi_selinv_ninv": [P, P, P, P, i32, f64, ctypes.c_int, P, P],
        "asi_selinv": [P, P, P, P, ctypes.c_int, P],
        "asi_ninv": [P, P, P, P, i32, f64, ctypes.c_int, P],
        "asi_mix": [P, P, P, f64, P],
        "asi_spai": [P, P, P, P, P, P, i32, P],
        "asi_lowrank": [P, i32, P, P, P, P],
        "asi_diag": [P, P, P],
        "asi_diag_err1": [P, P, P, i32, P, P, P],
        "asi_trace": [P, P, i32, P, P, P],
        "asi_ninv_full": [P, P, P, P, i32, f64, f64, i64, P, P, P, P],
        "asi_mix_full": [P, P, P, P, P, f64, i64, P, P, P, P],
        "asi_spmv": [P, P, P, P],
        "asi_ldl_solve": [P, P, P],
        "asi_pcg": [P, P, P, P, P, P, P, f64, i32, P, P],
        "asi_sqmr": [P, P, P, P, P, P, P, f64, i32, P, P],
        "asi_za_diag": [P, P, P, P, P, P, P],
        "asi_ildl_numeric": [P, P, P, P, P, P, P, P],
        "asi_check_matrix": [P, i32, P, P, P, P, f64],
        "asi_eigs_work_bytes": [i32, i32, i32, ctypes.POINTER(ctypes.c_size_t)],
        "asi_eigs_error": [P, P, P, P, P, P, P, i32, i32, i32, f64, i32, i32, f64, i32, P, ctypes.c_size_t, P, P, P,
                           P],
        "asi_block_solve_work_bytes": [i32, i32, ctypes.POINTER(ctypes.c_size_t)],
        "asi_pcg_block": [P, P, P, P, P, i32, P, P, f64, i32, P, ctypes.c_size_t, P, P],
        "asi_sqmr_block": [P, P, P, P, P, i32, P, P, f64, i32, P, ctypes.c_size_t, P, P],
        "asi_dense_symeig": [i32, P, P, P],
        "asi_sync": [P],
        "asi_profile": [P, ctypes.c_int],
        "asi_set_sweep": [P, ctypes.c_int],
        "asi_set_sentinel": [P, ctypes.c_int],
        "asi_sweep_plan": [P, P],
        "asi_unpermute": [P, P, P, P, P, P],
        "asi_unpermute_noalloc": [P, P, P, P, P, P],
        "asi_ildl_threshold_work_bytes": [i32, i32, i64, ctypes.POINTER(ctypes.c_size_t)],
        "asi_ildl_threshold": [P, i32, P, P, P, P, f64, i32, i32, i64, P, ctypes.c_size_t, ctypes.POINTER(i64),
                               P],
        "asi_ildl_threshold_extract": [P, P, P, P, P, P, P],
        "asi_mlp_features": [P, P, P, P, f64, P, P, P, P, P],
        "asi_mlp_pack": [P, P, P],
        "asi_mlp_forward": [P, P, P, i64, P],
        "asi_mlp_backward": [P, P, P, P, i64, P],
        "asi_mlp_loss": [P, P, P, i64, P, P],
        "asi_mlp_adam": [P, P, P, P, P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, i64],
        "asi_mlp_apply": [P, P, P, P, P],
        "asi_mlp_correct": [P, P, P, P, P, f64, P, P, P, P],
        "asi_mlp_correct_mix": [P, P, P, P, f64, P, P, P, P, P],
        "asi_profile_read": [P, i32, ctypes.POINTER(i64), ctypes.POINTER(f64), ctypes.POINTER(f64)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.asi_last_error.argtypes = [P]
    lib.asi_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Solver:
    """One handle of the library bound to a CUDA/HIP device of torch."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device("cuda", device)
        self.h = ctypes.c_void_p()
        self._check(self.lib.asi_create(ctypes.byref(self.h), device, None))
        self.ws = None
        self.n = 0
        self.nnzL = 0
        self.nnz_S = 0

    def __del__(self):
        try:
            if self.h:
                self.lib.asi_destroy(self.h)
        except Exception:
            pass

    # -- plumbing ------------------------------------------------------------
    def _check(self, rc):
        if rc != 0:
            msg = self.lib.asi_last_error(self.h) if self.h else b""
            raise AsiError(rc, (msg or b"").decode())

    def _stream(self):
        s = self.torch.cuda.current_stream(self.device)
        self._check(self.lib.asi_set_stream(self.h, ctypes.c_void_p(s.cuda_stream)))

    def _f64(self, x, n=None):
        t = self.torch.as_tensor(x, dtype=self.torch.float64, device=self.device).contiguous()
        if n is not None and t.numel() != n:
            raise ValueError(f"expected {n} entries, got {t.numel()}")
        return t

    # -- symbolic ------------------------------------------------------------
    def analyze(self, n, L_rowptr, L_col, piv, workspace_bytes=None, pool_entries=None):
        """asi_analyze + asi_set_workspace (the workspace is a torch uint8 tensor).

        ``pool_entries`` sizes the NInv pool (columns of L^inv, 20 bytes per
        entry); by default the library's suggestion is used.
        """
        rp = np.ascontiguousarray(L_rowptr, dtype=np.int64)
        cl = np.ascontiguousarray(L_col, dtype=np.int32)
        pv = np.ascontiguousarray(piv, dtype=np.int8)
        if len(cl) == 0:
            cl = np.zeros(1, np.int32)
        nnz = ctypes.c_int64()
        wsb = ctypes.c_size_t()
        self._check(self.lib.asi_analyze(self.h, int(n), rp.ctypes.data, cl.ctypes.data, pv.ctypes.data,
                                         ctypes.byref(nnz), ctypes.byref(wsb)))
        self.n = int(n)
        self.nnzL = int(rp[-1])
        self.nnz_S = int(nnz.value)
        if workspace_bytes is None and pool_entries is not None:
            workspace_bytes = self.info()["workspace_min"] + 20 * int(pool_entries) + 1024
        self.set_workspace(workspace_bytes or wsb.value)
        return self.nnz_S

    def set_workspace(self, nbytes):
        self.ws = self.torch.empty(int(nbytes) + 256, dtype=self.torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        aligned = (base + 255) & ~255
        self._stream()
        self._check(self.lib.asi_set_workspace(self.h, ctypes.c_void_p(aligned), int(nbytes)))

    def info(self):
        inf = Info()
        self._check(self.lib.asi_get_info(self.h, ctypes.byref(inf)))
        return inf.as_dict()

    def pattern(self, with_level=False):
        t = self.torch
        rp = t.empty(self.n + 1, dtype=t.int64, device=self.device)
        cl = t.empty(self.nnz_S, dtype=t.int32, device=self.device)
        lv = t.empty(self.n, dtype=t.int32, device=self.device) if with_level else None
        self._stream()
        self._check(self.lib.asi_get_pattern(self.h, _ptr(rp), _ptr(cl), _ptr(lv) if lv is not None else None))
        return (rp, cl, lv) if with_level else (rp, cl)

    # -- numeric -------------------------------------------------------------
    def _out(self, out):
        if out is None:
            return self.torch.empty(self.nnz_S, dtype=self.torch.float64, device=self.device)
        assert out.dtype == self.torch.float64 and out.numel() == self.nnz_S and out.is_contiguous()
        return out

    def load_factor(self, L_val, d_diag, d_sub):
        """asi_load_factor: later calls may pass None for the three factor arrays."""
        self._stream()
        self._check(self.lib.asi_load_factor(self.h, _ptr(L_val), _ptr(d_diag), _ptr(d_sub)))

    def selinv(self, L_val=None, d_diag=None, d_sub=None, precision="fp64", out=None):
        out = self._out(out)
        self._stream()
        self._check(self.lib.asi_selinv(self.h, _ptr(L_val), _ptr(d_diag), _ptr(d_sub),
                                        PRECISION[precision], _ptr(out)))
        return out

    def selinv_ninv(self, L_val=None, d_diag=None, d_sub=None, p=3, delta=0.1, precision="fp64",
                    Z=None, N=None):
        """SelInv and NInv concurrently (NInv on the handle's second stream); returns (Z, N)."""
        Z = self._out(Z)
        N = self._out(N)
        self._stream()
        self._check(self.lib.asi_selinv_ninv(self.h, _ptr(L_val), _ptr(d_diag), _ptr(d_sub), int(p),
                                             float(delta), PRECISION[precision], _ptr(Z), _ptr(N)))
        return Z, N

    def ninv(self, L_val=None, d_diag=None, d_sub=None, p=3, delta=0.1, precision="fp64", out=None):
        out = self._out(out)
        self._stream()
        self._check(self.lib.asi_ninv(self.h, _ptr(L_val), _ptr(d_diag), _ptr(d_sub), int(p),
                                      float(delta), PRECISION[precision], _ptr(out)))
        return out

    def mix(self, Z, N, eps=1e-2, out=None):
        out = self._out(out)
        self._stream()
        self._check(self.lib.asi_mix(self.h, _ptr(Z), _ptr(N), float(eps), _ptr(out)))
        return out

    def spai(self, A_rowptr, A_col, A_val, perm, M, cg_iters=10, out=None):
        out = self._out(out)
        self._stream()
        self._check(self.lib.asi_spai(self.h, _ptr(A_rowptr), _ptr(A_col), _ptr(A_val), _ptr(perm),
                                      _ptr(M), int(cg_iters), _ptr(out)))
        return out

    def lowrank(self, V, lam, X, out=None):
        out = self._out(out)
        self._stream()
        k = int(V.shape[1])
        self._check(self.lib.asi_lowrank(self.h, k, _ptr(V), _ptr(lam), _ptr(X), _ptr(out)))
        return out

    # -- learned correction --------------------------------------------------
    def mlp_features(self, Z, N, M, eps, L_val=None, d_diag=None, d_sub=None, F=None, sc=None):
        """(features |S| x 16 as int16 bfloat16 words, scale |S| float32)."""
        t = self.torch
        if F is None:
            F = t.empty((self.nnz_S, MLP_FEATURES), dtype=t.int16, device=self.device)
        if sc is None:
            sc = t.empty(self.nnz_S, dtype=t.float32, device=self.device)
        self._stream()
        self._check(self.lib.asi_mlp_features(self.h, _ptr(Z), _ptr(N), _ptr(M), float(eps), _ptr(L_val),
                                              _ptr(d_diag), _ptr(d_sub), _ptr(F), _ptr(sc)))
        return F, sc

    def mlp_pack(self, theta, packed=None):
        t = self.torch
        if packed is None:
            packed = t.empty(MLP_PACKED_BYTES, dtype=t.uint8, device=self.device)
        self._stream()
        self._check(self.lib.asi_mlp_pack(self.h, _ptr(theta), _ptr(packed)))
        return packed

    def mlp_forward(self, packed, F, rows=None, y=None):
        t = self.torch
        rows = F.shape[0] if rows is None else int(rows)
        if y is None:
            y = t.empty(rows, dtype=t.float32, device=self.device)
        self._stream()
        self._check(self.lib.asi_mlp_forward(self.h, _ptr(packed), _ptr(F), rows, _ptr(y)))
        return y

    def mlp_backward(self, packed, F, dy, grad, rows=None):
        rows = F.shape[0] if rows is None else int(rows)
        self._stream()
        self._check(self.lib.asi_mlp_backward(self.h, _ptr(packed), _ptr(F), _ptr(dy), rows, _ptr(grad)))
        return grad

    def mlp_loss(self, y, target, dy, loss, rows=None):
        rows = y.shape[0] if rows is None else int(rows)
        self._stream()
        self._check(self.lib.asi_mlp_loss(self.h, _ptr(y), _ptr(target), rows, _ptr(dy), _ptr(loss)))
        return dy

    def mlp_adam(self, theta, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self._stream()
        self._check(self.lib.asi_mlp_adam(self.h, _ptr(theta), _ptr(m), _ptr(v), _ptr(grad), float(lr),
                                          float(beta1), float(beta2), float(eps), int(step)))

    def mlp_apply(self, M, y, scale, out=None):
        out = self._out(out)
        self._stream()
        self._check(self.lib.asi_mlp_apply(self.h, _ptr(M), _ptr(y), _ptr(scale), _ptr(out)))
        return out

    def mlp_correct(self, packed, Z, N, M, eps, L_val=None, d_diag=None, d_sub=None, out=None):
        """M + y s on S from features, network and correction in one pass."""
        out = self._out(out)
        self._stream()
        self._check(self.lib.asi_mlp_correct(self.h, _ptr(packed), _ptr(Z), _ptr(N), _ptr(M), float(eps),
                                             _ptr(L_val), _ptr(d_diag), _ptr(d_sub), _ptr(out)))
        return out

    def mlp_correct_mix(self, packed, Z, N, eps, L_val=None, d_diag=None, d_sub=None, M=None, out=None):
        """Mix and the learned correction in one pass: returns out = M + y s
        (and writes M = Mix(Z, N) into M when given)."""
        out = self._out(out)
        self._stream()
        self._check(self.lib.asi_mlp_correct_mix(self.h, _ptr(packed), _ptr(Z), _ptr(N), float(eps), _ptr(L_val),
                                                 _ptr(d_diag), _ptr(d_sub), _ptr(M), _ptr(out)))
        return out

    def diag(self, X, out=None):
        t = self.torch
        if out is None:
            out = t.empty(self.n, dtype=t.float64, device=self.device)
        self._stream()
        self._check(self.lib.asi_diag(self.h, _ptr(X), _ptr(out)))
        return out

    def diag_err1(self, d_ref, d_hat, V=None, lam=None, sums=None):
        """Device float64[2]: (sum |d_ref - d_hat - sum_m lam_m V_im^2|, sum |d_ref|)."""
        t = self.torch
        if sums is None:
            sums = t.empty(2, dtype=t.float64, device=self.device)
        k = 0 if V is None else int(V.shape[1])
        self._stream()
        self._check(self.lib.asi_diag_err1(self.h, _ptr(d_ref), _ptr(d_hat), k,
                                           _ptr(V) if k else None, _ptr(lam) if k else None, _ptr(sums)))
        return sums

    def _full_call(self, fn, args):
        """Two-pass call of a full-pattern entry point: size, allocate, fill."""
        t = self.torch
        nnz = ctypes.c_int64(0)
        rowptr = t.empty(self.n + 1, dtype=t.int64, device=self.device)
        self._stream()
        rc = fn(self.h, *args, 0, _ptr(rowptr), None, None, ctypes.byref(nnz))
        if rc != 0 and nnz.value == 0:
            self._check(rc)
        col = t.empty(max(nnz.value, 1), dtype=t.int32, device=self.device)
        val = t.empty(max(nnz.value, 1), dtype=t.float64, device=self.device)
        self._check(fn(self.h, *args, nnz.value, _ptr(rowptr), _ptr(col), _ptr(val), ctypes.byref(nnz)))
        return rowptr, col[:nnz.value], val[:nnz.value]

    def ninv_full(self, L_val=None, d_diag=None, d_sub=None, p=3, delta=0.1, drop=0.1):
        """NInv on its own pattern: lower triangle as (rowptr int64, col int32, val float64)."""
        return self._full_call(self.lib.asi_ninv_full, (_ptr(L_val), _ptr(d_diag), _ptr(d_sub), int(p),
                                                        float(delta), float(drop)))

    def mix_full(self, Z, N_full, eps=1e-2):
        """Mix on NInv's pattern joined with S_eps: lower triangle as (rowptr, col, val)."""
        rp, cl, vl = N_full
        return self._full_call(self.lib.asi_mix_full, (_ptr(Z), _ptr(rp), _ptr(cl), _ptr(vl), float(eps)))

    def ildl_numeric(self, A_rowptr, A_col, A_val, perm, L_val=None, d_diag=None, d_sub=None):
        """Numeric phase of the incomplete factorization on the analysed
        pattern and pivots (device): returns (L_val, d_diag, d_sub), ready for
        load_factor. A is the device CSR of A in its own ordering."""
        t = self.torch
        f = lambda x, m: t.empty(m, dtype=t.float64, device=self.device) if x is None else x
        L_val, d_diag, d_sub = f(L_val, max(self.nnzL, 1)), f(d_diag, self.n), f(d_sub, self.n)
        self._stream()
        self._check(self.lib.asi_ildl_numeric(self.h, _ptr(A_rowptr), _ptr(A_col), _ptr(A_val), _ptr(perm),
                                              _ptr(L_val), _ptr(d_diag), _ptr(d_sub)))
        return L_val, d_diag, d_sub

    def ildl_threshold(self, A_rowptr, A_col, A_val, q, tau, pivoting=True, row_cap=512, pool_cap=None,
                       max_retries=6):
        """The threshold incomplete factorization on the device (asi_ildl_threshold
        and _extract). A: device CSR in its own ordering; q: the ordering.
        Returns (L_rowptr, L_col, L_val, d_diag, d_sub, piv) device tensors and
        stats {rounds, replaced_pivots, row_cap, pool_cap}. row_cap and
        pool_cap (default 64 n) are doubled and the call repeated when the
        library reports them too small."""
        t = self.torch
        n = int(A_rowptr.numel()) - 1
        q = t.as_tensor(q, dtype=t.int32, device=self.device).contiguous()
        pool_cap = int(pool_cap) if pool_cap is not None else 64 * n
        for attempt in range(max_retries + 1):
            nbytes = ctypes.c_size_t(0)
            self._check(self.lib.asi_ildl_threshold_work_bytes(n, int(row_cap), int(pool_cap),
                                                               ctypes.byref(nbytes)))
            work = t.empty(nbytes.value + 256, dtype=t.uint8, device=self.device)
            base = (work.data_ptr() + 255) & ~255
            nnz = ctypes.c_int64(0)
            stats = np.zeros(2, np.int64)
            self._stream()
            rc = self.lib.asi_ildl_threshold(self.h, n, _ptr(A_rowptr), _ptr(A_col), _ptr(A_val), _ptr(q),
                                             float(tau), 1 if pivoting else 0, int(row_cap), int(pool_cap),
                                             ctypes.c_void_p(base), nbytes.value, ctypes.byref(nnz),
                                             stats.ctypes.data)
            if rc == 6 and attempt < max_retries:  # ASI_E_WORKSPACE: a cap was too small
                del work
                row_cap, pool_cap = 2 * int(row_cap), 2 * int(pool_cap)
                continue
            self._check(rc)
            break
        m = int(nnz.value)
        Lp = t.empty(n + 1, dtype=t.int64, device=self.device)
        Lc = t.empty(max(m, 1), dtype=t.int32, device=self.device)
        Lv = t.empty(max(m, 1), dtype=t.float64, device=self.device)
        dd = t.empty(n, dtype=t.float64, device=self.device)
        ds = t.empty(n, dtype=t.float64, device=self.device)
        pv = t.empty(n, dtype=t.int8, device=self.device)
        self._check(self.lib.asi_ildl_threshold_extract(self.h, _ptr(Lp), _ptr(Lc), _ptr(Lv), _ptr(dd), _ptr(ds),
                                                        _ptr(pv)))
        self.sync()
        del work
        return (Lp, Lc[:m], Lv[:m], dd, ds, pv), {"rounds": int(stats[0]), "replaced_pivots": int(stats[1]),
                                                  "row_cap": int(row_cap), "pool_cap": int(pool_cap)}

    def unpermute(self, perm, X):
        """Values X on S (factor ordering) as a CSR matrix in A's ordering:
        (rowptr int64, col int32, val float64) device tensors, row perm[i]
        holding row i of S with columns renamed by perm and sorted."""
        t = self.torch
        perm = t.as_tensor(perm, dtype=t.int32, device=self.device).contiguous()
        rp = t.empty(self.n + 1, dtype=t.int64, device=self.device)
        cl = t.empty(self.nnz_S, dtype=t.int32, device=self.device)
        vl = t.empty(self.nnz_S, dtype=t.float64, device=self.device)
        self._stream()
        self._check(self.lib.asi_unpermute(self.h, _ptr(perm), _ptr(X), _ptr(rp), _ptr(cl), _ptr(vl)))
        return rp, cl, vl

    def za_diag(self, A_rowptr, A_col, A_val, perm, Z, d=None):
        """Device float64[n]: (Z Ah)_ii, Ah = P^T A P."""
        t = self.torch
        d = t.empty(self.n, dtype=t.float64, device=self.device) if d is None else d
        self._stream()
        self._check(self.lib.asi_za_diag(self.h, _ptr(A_rowptr), _ptr(A_col), _ptr(A_val), _ptr(perm), _ptr(Z),
                                         _ptr(d)))
        return d

    def check_matrix(self, A, perm=None, tol=0.0):
        """Host check of a scipy CSR A (and perm): raises AsiError on invalid input."""
        indptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
        indices = np.ascontiguousarray(A.indices, dtype=np.int32)
        data = np.ascontiguousarray(A.data, dtype=np.float64)
        pp = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
        c = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
        self._check(self.lib.asi_check_matrix(self.h, int(A.shape[0]), c(indptr), c(indices), c(data), c(pp),
                                              float(tol)))

    def spmv(self, X, x, y=None):
        """y = X x for X on S."""
        y = self.torch.empty_like(x) if y is None else y
        self._stream()
        self._check(self.lib.asi_spmv(self.h, _ptr(X), _ptr(x), _ptr(y)))
        return y

    def ldl_solve(self, x, y=None):
        """y = (L D L^T)^-1 x with the loaded factor."""
        y = self.torch.empty_like(x) if y is None else y
        self._stream()
        self._check(self.lib.asi_ldl_solve(self.h, _ptr(x), _ptr(y)))
        return y

    def _krylov(self, fn, A_rowptr, A_col, A_val, perm, b, x, tol, maxit):
        x = self.torch.empty_like(b) if x is None else x
        it = ctypes.c_int32(0)
        rr = ctypes.c_double(0.0)
        self._stream()
        self._check(fn(self.h, _ptr(A_rowptr), _ptr(A_col), _ptr(A_val), _ptr(perm), _ptr(b), _ptr(x), float(tol),
                       int(maxit), ctypes.byref(it), ctypes.byref(rr)))
        return x, it.value, rr.value

    def pcg(self, A_rowptr, A_col, A_val, perm, b, x=None, tol=1e-10, maxit=1000):
        """x = Ah^-1 b by CG preconditioned with the loaded factor; returns (x, steps, relres)."""
        return self._krylov(self.lib.asi_pcg, A_rowptr, A_col, A_val, perm, b, x, tol, maxit)

    def sqmr(self, A_rowptr, A_col, A_val, perm, b, x=None, tol=1e-10, maxit=1000):
        """x = Ah^-1 b by simplified QMR preconditioned with the loaded factor; returns (x, steps, relres)."""
        return self._krylov(self.lib.asi_sqmr, A_rowptr, A_col, A_val, perm, b, x, tol, maxit)

    def eigs_error(self, A_rowptr, A_col, A_val, perm, X, k, m=None, block=1, v0=None, seed=0, tol=1e-8,
                   max_restarts=200, method="cg", solve_tol=1e-12, solve_maxit=1000, work=None):
        """k eigenpairs of E = A^-1 - X of largest |lambda| by the device
        (block) Lanczos iteration (A^-1 by block PCG, method "cg", or block
        SQMR, "sqmr"). m defaults to min(max(2k + 1, 20) + block - 1, 256,
        n - block); v0 (device float64 [block, n], row v = start vector v)
        defaults to standard normal vectors drawn with numpy from seed.
        Returns (lam numpy[k], V device [n, k] row-major, estimated relative
        residuals numpy[k], stats dict)."""
        t = self.torch
        n = self.n
        b = int(block)
        m = int(m) if m is not None else min(max(2 * k + 1, 20) + b - 1, 256, n - b)
        if v0 is None:
            v0 = t.as_tensor(np.random.default_rng(seed).standard_normal((b, n)), device=self.device)
        nbytes = ctypes.c_size_t(0)
        self._check(self.lib.asi_eigs_work_bytes(n, m, b, ctypes.byref(nbytes)))
        if work is None or work.numel() * work.element_size() < nbytes.value:
            work = t.empty((nbytes.value + 7) // 8, dtype=t.float64, device=self.device)
        lam = np.zeros(k)
        res = np.zeros(k)
        stats = np.zeros(5)
        V = t.empty((n, k), dtype=t.float64, device=self.device)
        c = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        self._stream()
        self._check(self.lib.asi_eigs_error(
            self.h, _ptr(A_rowptr), _ptr(A_col), _ptr(A_val), _ptr(perm), _ptr(X), _ptr(v0), int(k), m, b,
            float(tol), int(max_restarts), {"cg": 0, "sqmr": 1}[method], float(solve_tol), int(solve_maxit),
            _ptr(work), work.numel() * work.element_size(), c(lam), _ptr(V), c(res), c(stats)))
        names = ["applications", "krylov_steps", "restarts", "converged", "max_solve_relres"]
        st = {a: (float(b_) if a == "max_solve_relres" else int(b_)) for a, b_ in zip(names, stats)}
        st["m"] = m
        st["block"] = b
        return lam, V, res, st

    def _block_solve(self, fn, A_rowptr, A_col, A_val, perm, B, X, tol, maxit):
        t = self.torch
        nrhs = int(B.shape[0])
        X = t.empty_like(B) if X is None else X
        nbytes = ctypes.c_size_t(0)
        self._check(self.lib.asi_block_solve_work_bytes(self.n, nrhs, ctypes.byref(nbytes)))
        work = t.empty((nbytes.value + 7) // 8, dtype=t.float64, device=self.device)
        iters = np.zeros(nrhs, dtype=np.int32)
        rel = np.zeros(nrhs)
        c = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        self._stream()
        self._check(fn(self.h, _ptr(A_rowptr), _ptr(A_col), _ptr(A_val), _ptr(perm), nrhs, _ptr(B), _ptr(X),
                       float(tol), int(maxit), _ptr(work), work.numel() * 8, c(iters), c(rel)))
        return X, iters, rel

    def pcg_block(self, A_rowptr, A_col, A_val, perm, B, X=None, tol=1e-10, maxit=1000):
        """Block PCG: B, X device float64 [nrhs, n] (row v = vector v); returns (X, iters, relres)."""
        return self._block_solve(self.lib.asi_pcg_block, A_rowptr, A_col, A_val, perm, B, X, tol, maxit)

    def sqmr_block(self, A_rowptr, A_col, A_val, perm, B, X=None, tol=1e-10, maxit=1000):
        """Block SQMR: B, X device float64 [nrhs, n]; returns (X, iters, relres)."""
        return self._block_solve(self.lib.asi_sqmr_block, A_rowptr, A_col, A_val, perm, B, X, tol, maxit)

    def trace(self, X, V=None, lam=None, sums=None):
        """Device float64[2]: (sum_i c_i, sum_i |c_i|), c_i = X_ii + sum_m lam_m V_im^2."""
        t = self.torch
        if sums is None:
            sums = t.empty(2, dtype=t.float64, device=self.device)
        k = 0 if V is None else int(V.shape[1])
        self._stream()
        self._check(self.lib.asi_trace(self.h, _ptr(X), k, _ptr(V) if k else None, _ptr(lam) if k else None,
                                       _ptr(sums)))
        return sums

    def sync(self):
        self._stream()
        self._check(self.lib.asi_sync(self.h))

    def set_sweep(self, mode="auto"):
        """SelInv schedule: "auto", "levels" (one launch per DAG level) or "dataflow"."""
        self._check(self.lib.asi_set_sweep(self.h, SWEEP[mode]))

    def set_sentinel(self, on=True):
        """Schedule check: SelInv sweeps start from a NaN-filled working Z, so
        a read of an entry before its block writes it shows up as a
        non-finite result."""
        self._check(self.lib.asi_set_sentinel(self.h, 1 if on else 0))

    def sweep_plan(self):
        """{variant: level launches per SelInv sweep} of the level schedule."""
        counts = np.zeros(len(SWEEP_VARIANTS), np.int64)
        self._check(self.lib.asi_sweep_plan(self.h, counts.ctypes.data))
        return dict(zip(SWEEP_VARIANTS, (int(c) for c in counts)))

    def profile(self, enable=True):
        self._stream()
        self._check(self.lib.asi_profile(self.h, 1 if enable else 0))

    def profile_read(self):
        """{class: (launches, total_ms, algorithmic_bytes)} for every kernel class."""
        out = {}
        for name, k in KERNEL_CLASSES.items():
            n = ctypes.c_int64()
            ms = ctypes.c_double()
            b = ctypes.c_double()
            self._check(self.lib.asi_profile_read(self.h, k, ctypes.byref(n), ctypes.byref(ms),
                                                  ctypes.byref(b)))
            out[name] = (n.value, ms.value, b.value)
        return out


def dense_symeig(T):
    """All eigenpairs of a small dense symmetric matrix with the library's
    host Jacobi routine (the Lanczos iteration's projected problem): returns
    (theta ascending, Y with unit eigenvectors as columns)."""
    lib = load_library()
    T = np.ascontiguousarray(T, dtype=np.float64)
    m = T.shape[0]
    if T.ndim != 2 or T.shape[1] != m:
        raise ValueError("T must be square")
    theta = np.empty(m)
    Y = np.empty((m, m))
    c = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    rc = lib.asi_dense_symeig(m, c(T), c(theta), c(Y))
    if rc != 0:
        raise AsiError(rc, "asi_dense_symeig failed")
    return theta, Y


def upload_factors(F, device="cuda:0"):
    """Device copies of the numeric factor arrays (L values, D) as torch tensors."""
    import torch
    dev = torch.device(device)
    return (torch.as_tensor(F.L_val, dtype=torch.float64, device=dev),
            torch.as_tensor(F.d_diag, dtype=torch.float64, device=dev),
            torch.as_tensor(F.d_sub, dtype=torch.float64, device=dev))
