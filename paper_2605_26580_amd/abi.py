"""ctypes binding of libcider.so: the C ABI of include/cider.h, same names.

Only argument marshalling lives here: torch tensors are passed as device
pointers, the current torch stream as the HIP stream.  Every step of the
decoder runs inside the HIP library; if the library is missing the first
call raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Tuple, Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcider.so")

CIDER_OK, CIDER_EINVAL, CIDER_ENOMEM, CIDER_EDEVICE, CIDER_EUNSUPPORTED, CIDER_EAGAIN = 0, -1, -2, -3, -4, -5
CIDER_FP32, CIDER_BF16, CIDER_FP8, CIDER_FP64 = 0, 1, 2, 3
CIDER_SCHED_LINEAR, CIDER_SCHED_COSINE = 0, 1
CIDER_MASK = 2

EXPORTS = [
    "cider_opts_default", "cider_weights_blob_floats", "cider_weights_create", "cider_weights_destroy",
    "cider_code_create", "cider_code_destroy", "cider_workspace_size", "cider_decode",
    "cider_decode_batch", "cider_decode_noalloc", "cider_step_debug", "cider_evidence", "cider_amp_evidence", "cider_gf64_check_update", "cider_server_create",
    "cider_server_submit", "cider_server_poll", "cider_server_drain", "cider_server_destroy",
    "cider_strerror", "cider_last_error", "cider_profile_read", "cider_tuning_read",
    "cider_code_create_q", "cider_decode_q_batch", "cider_step_debug_q", "cider_server_budget_floor",
]


class CiderError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str):
        super().__init__(f"{what} failed: {detail or 'status ' + str(status)} (status {status})")
        self.status = status


class cider_model_cfg(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("d", C.c_int32), ("heads", C.c_int32),
                ("mlp_mult", C.c_int32), ("n_max", C.c_int32), ("q", C.c_int32)]


class cider_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("schedule", C.c_int32), ("first_reveal", C.c_int32),
                ("remask", C.c_int32), ("remask_max_rounds", C.c_int32), ("final_argmax", C.c_int32),
                ("use_graph", C.c_int32), ("remask_thr", C.c_float), ("tau", C.c_float),
                ("eta", C.c_float), ("lam_max", C.c_float), ("lam_min", C.c_float),
                ("tau_max", C.c_float), ("tau_min", C.c_float),
                ("autotune", C.c_int32), ("profile", C.c_int32), ("fused_blocks", C.c_int32),
                ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t),
                ("qhead", C.c_void_p), ("qhead_hidden", C.c_int32), ("remask_stages", C.c_int32),
                ("remask_phi", C.c_float * 4)]


class cider_bin(C.Structure):
    _fields_ = [("y", C.c_void_p), ("sigma2", C.c_float), ("code", C.c_void_p), ("K", C.c_int32),
                ("n", C.c_int32), ("out_symbols", C.c_void_p), ("out_logits", C.c_void_p),
                ("out_row_valid", C.c_void_p), ("out_rounds", C.c_void_p)]


class cider_qbin(C.Structure):
    _fields_ = [("S", C.c_void_p), ("code", C.c_void_p), ("K", C.c_int32), ("n", C.c_int32),
                ("out_symbols", C.c_void_p), ("out_logits", C.c_void_p), ("out_row_valid", C.c_void_p)]


class cider_kernel_stat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("total_ms", C.c_double)]


class cider_tuning_entry(C.Structure):
    _fields_ = [("role", C.c_char * 24), ("n", C.c_int32), ("kd", C.c_int32), ("bucket", C.c_int32),
                ("tile", C.c_int32), ("best_ms", C.c_double), ("default_ms", C.c_double)]


class cider_server_cfg(C.Structure):
    _fields_ = [("weights", C.c_void_p), ("opts", cider_opts), ("steps", C.c_int32),
                ("max_slots", C.c_int32), ("max_queue", C.c_int32), ("hbm_budget", C.c_size_t),
                ("max_tokens", C.c_int64)]


class cider_result(C.Structure):
    _fields_ = [("id", C.c_uint64), ("K", C.c_int32), ("n", C.c_int32), ("status", C.c_int32),
                ("rounds", C.c_int32), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double)]


_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    """Load libcider.so (built by paper_2605_26580_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built; run paper_2605_26580_amd.build.build()")
    # torch first: the library then binds to the HIP runtime torch has already
    # loaded, so the process holds one runtime.  Loaded the other way round,
    # two runtimes end up in the process and the second to start sees no device.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, f32 = C.c_void_p, C.c_int32, C.c_float
    L.cider_opts_default.argtypes = [C.POINTER(cider_opts)]
    L.cider_opts_default.restype = None
    L.cider_weights_blob_floats.argtypes = [C.POINTER(cider_model_cfg)]
    L.cider_weights_blob_floats.restype = C.c_size_t
    L.cider_weights_create.argtypes = [C.POINTER(cider_model_cfg), vp, C.c_size_t, C.POINTER(vp)]
    L.cider_weights_destroy.argtypes = [vp]
    L.cider_weights_destroy.restype = None
    L.cider_code_create.argtypes = [i32, i32, vp, vp, C.POINTER(vp)]
    L.cider_code_destroy.argtypes = [vp]
    L.cider_code_create_q.argtypes = [i32, i32, vp, vp, vp, i32, C.POINTER(vp)]
    L.cider_decode_q_batch.argtypes = [i32, C.POINTER(cider_qbin), vp, i32, C.POINTER(cider_opts), vp]
    L.cider_step_debug_q.argtypes = [vp, vp, vp, vp, i32, i32, vp, f32, i32, i32, C.POINTER(cider_opts),
                                     vp, vp, vp]
    L.cider_code_destroy.restype = None
    L.cider_workspace_size.argtypes = [vp, i32, C.c_int64, C.c_int64, C.POINTER(cider_opts),
                                       C.POINTER(C.c_size_t)]
    L.cider_decode.argtypes = [vp, f32, vp, i32, i32, vp, i32, vp, C.POINTER(cider_opts), vp]
    L.cider_decode_noalloc.argtypes = [vp, f32, vp, i32, i32, vp, i32, vp, C.POINTER(cider_opts), vp]
    L.cider_decode_batch.argtypes = [i32, C.POINTER(cider_bin), vp, i32, C.POINTER(cider_opts), vp]
    L.cider_step_debug.argtypes = [vp, vp, vp, f32, vp, i32, i32, vp, f32, i32, i32,
                                   C.POINTER(cider_opts), vp, vp, vp, vp]
    L.cider_evidence.argtypes = [vp, f32, i32, i32, vp, vp, vp]
    L.cider_amp_evidence.argtypes = [vp, vp, C.c_int64, i32, i32, f32, f32, i32, vp, vp]
    L.cider_gf64_check_update.argtypes = [vp, vp, vp, C.c_int64, C.c_int64, vp, vp]
    L.cider_server_create.argtypes = [C.POINTER(cider_server_cfg), C.POINTER(vp)]
    L.cider_server_submit.argtypes = [vp, vp, f32, vp, i32, i32, vp, C.POINTER(C.c_uint64)]
    L.cider_server_poll.argtypes = [vp, C.POINTER(cider_result), i32, C.POINTER(i32)]
    L.cider_server_drain.argtypes = [vp]
    L.cider_server_budget_floor.argtypes = [C.POINTER(cider_server_cfg), C.POINTER(C.c_size_t)]
    L.cider_server_destroy.argtypes = [vp]
    L.cider_server_destroy.restype = None
    L.cider_profile_read.argtypes = [vp, C.POINTER(cider_kernel_stat), i32, C.POINTER(i32), i32]
    L.cider_tuning_read.argtypes = [vp, C.POINTER(cider_tuning_entry), i32, C.POINTER(i32)]
    L.cider_strerror.argtypes = [C.c_int]
    L.cider_strerror.restype = C.c_char_p
    L.cider_last_error.argtypes = []
    L.cider_last_error.restype = C.c_char_p
    for name in ("cider_weights_create", "cider_code_create", "cider_workspace_size", "cider_decode",
                 "cider_decode_batch", "cider_decode_noalloc", "cider_step_debug", "cider_evidence", "cider_amp_evidence", "cider_gf64_check_update",
                 "cider_server_create", "cider_server_submit", "cider_server_poll", "cider_server_drain",
                 "cider_profile_read", "cider_tuning_read"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(status: int, what: str) -> None:
    if status != CIDER_OK:
        detail = lib().cider_last_error().decode(errors="replace")
        raise CiderError(status, what, detail)


# ---- helpers ---------------------------------------------------------------

def _ptr(t) -> Optional[int]:
    """Device pointer of a contiguous torch tensor (None passes NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream(stream=None) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream or None


def cider_opts_default(**overrides) -> cider_opts:
    o = cider_opts()
    lib().cider_opts_default(C.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        if k == "remask_phi":
            v = (C.c_float * 4)(*(list(v) + [0.0] * (4 - len(v))))
        elif k == "qhead" and v is not None and not isinstance(v, int):
            v = _ptr(v)
        setattr(o, k, v)
    return o


def make_cfg(n_layers: int, d: int, heads: int, mlp_mult: int = 4, n_max: int = 1024, q: int = 0) -> cider_model_cfg:
    return cider_model_cfg(n_layers, d, heads, mlp_mult, n_max, q)


def cider_weights_blob_floats(cfg: cider_model_cfg) -> int:
    return int(lib().cider_weights_blob_floats(C.byref(cfg)))


class Weights:
    """Owns a cider_weights handle (device copies of the model)."""

    def __init__(self, cfg: cider_model_cfg, blob: np.ndarray):
        blob = np.ascontiguousarray(blob, dtype=np.float32)
        h = C.c_void_p()
        check(lib().cider_weights_create(C.byref(cfg), blob.ctypes.data, blob.size, C.byref(h)),
              "cider_weights_create")
        self.cfg = cfg
        self.handle = h

    def close(self):
        if self.handle:
            lib().cider_weights_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cider_weights_create(cfg: cider_model_cfg, blob: np.ndarray) -> Weights:
    return Weights(cfg, blob)


class Code:
    """Owns a cider_code handle (binary H as CSR on the device)."""

    def __init__(self, n: int, m: int, row_ptr: np.ndarray, col_idx: np.ndarray):
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        h = C.c_void_p()
        check(lib().cider_code_create(int(n), int(m), rp.ctypes.data, ci.ctypes.data, C.byref(h)),
              "cider_code_create")
        self.n, self.m = int(n), int(m)
        self.handle = h

    def close(self):
        if self.handle:
            lib().cider_code_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cider_code_create(n: int, m: int, row_ptr, col_idx) -> Code:
    return Code(n, m, row_ptr, col_idx)


class CodeQ(Code):
    """Owns a cider_code handle of a GF(2^q_bits) code (CSR plus edge coefficients)."""

    def __init__(self, n: int, m: int, row_ptr: np.ndarray, col_idx: np.ndarray, coef: np.ndarray, q_bits: int):
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        cf = np.ascontiguousarray(coef, dtype=np.uint8)
        h = C.c_void_p()
        check(lib().cider_code_create_q(int(n), int(m), rp.ctypes.data, ci.ctypes.data, cf.ctypes.data,
                                        int(q_bits), C.byref(h)), "cider_code_create_q")
        self.n, self.m, self.q_bits = int(n), int(m), int(q_bits)
        self.handle = h


def cider_code_create_q(n: int, m: int, row_ptr, col_idx, coef, q_bits: int) -> CodeQ:
    return CodeQ(n, m, row_ptr, col_idx, coef, q_bits)


def cider_decode_q_batch(bins: Sequence[dict], w: Weights, steps: int, opts: Optional[cider_opts] = None,
                         stream=None) -> None:
    """bins: dicts with S, code, K, n, out_symbols and optional out_logits, out_row_valid."""
    arr = (cider_qbin * len(bins))()
    for i, b in enumerate(bins):
        arr[i] = cider_qbin(_ptr(b["S"]), b["code"].handle, int(b["K"]), int(b["n"]), _ptr(b["out_symbols"]),
                            _ptr(b.get("out_logits")), _ptr(b.get("out_row_valid")))
    check(lib().cider_decode_q_batch(len(bins), arr, w.handle, steps, C.byref(opts) if opts is not None else None,
                                     _stream(stream)), "cider_decode_q_batch")


def cider_step_debug_q(X_in, X_out, S, code: Code, K: int, n: int, w: Weights, gamma: float, reveal_count: int,
                       first: int, opts: Optional[cider_opts] = None, out_lbar=None, out_logits=None,
                       stream=None) -> None:
    check(lib().cider_step_debug_q(_ptr(X_in), _ptr(X_out), _ptr(S), code.handle, K, n, w.handle, float(gamma),
                                   int(reveal_count), int(first), C.byref(opts) if opts is not None else None,
                                   _ptr(out_lbar), _ptr(out_logits), _stream(stream)), "cider_step_debug_q")


def cider_workspace_size(w: Weights, num_bins: int, total_tokens: int, total_slots: int,
                         opts: Optional[cider_opts] = None) -> int:
    out = C.c_size_t()
    check(lib().cider_workspace_size(w.handle, num_bins, total_tokens, total_slots,
                                     C.byref(opts) if opts is not None else None, C.byref(out)),
          "cider_workspace_size")
    return int(out.value)


def cider_decode(y, sigma2: float, code: Code, K: int, n: int, w: Weights, steps: int, out_symbols,
                 opts: Optional[cider_opts] = None, stream=None) -> None:
    check(lib().cider_decode(_ptr(y), float(sigma2), code.handle, K, n, w.handle, steps, _ptr(out_symbols),
                             C.byref(opts) if opts is not None else None, _stream(stream)), "cider_decode")


def cider_decode_noalloc(y, sigma2: float, code: Code, K: int, n: int, w: Weights, steps: int, out_symbols,
                         opts: Optional[cider_opts] = None, stream=None) -> None:
    check(lib().cider_decode_noalloc(_ptr(y), float(sigma2), code.handle, K, n, w.handle, steps,
                                     _ptr(out_symbols), C.byref(opts) if opts is not None else None,
                                     _stream(stream)), "cider_decode_noalloc")


def cider_decode_batch(bins: Sequence[dict], w: Weights, steps: int, opts: Optional[cider_opts] = None,
                       stream=None) -> None:
    """bins: dicts with y, sigma2, code, K, n, out_symbols and optional out_logits, out_row_valid,
    out_rounds."""
    arr = (cider_bin * len(bins))()
    for i, b in enumerate(bins):
        arr[i] = cider_bin(_ptr(b["y"]), float(b["sigma2"]), b["code"].handle, int(b["K"]), int(b["n"]),
                           _ptr(b["out_symbols"]), _ptr(b.get("out_logits")), _ptr(b.get("out_row_valid")),
                           _ptr(b.get("out_rounds")))
    check(lib().cider_decode_batch(len(bins), arr, w.handle, steps, C.byref(opts) if opts is not None else None,
                                   _stream(stream)), "cider_decode_batch")


def cider_step_debug(X_in, X_out, y, sigma2: float, code: Code, K: int, n: int, w: Weights, gamma: float,
                     reveal_count: int, first: int, opts: Optional[cider_opts] = None, out_lbar=None,
                     out_logits=None, out_z=None, stream=None) -> None:
    check(lib().cider_step_debug(_ptr(X_in), _ptr(X_out), _ptr(y), float(sigma2), code.handle, K, n, w.handle,
                                 float(gamma), int(reveal_count), int(first),
                                 C.byref(opts) if opts is not None else None, _ptr(out_lbar), _ptr(out_logits),
                                 _ptr(out_z), _stream(stream)), "cider_step_debug")


def cider_gf64_check_update(p_edge, row_ptr, coef, checks: int, edges: int, out_msg, stream=None) -> None:
    check(lib().cider_gf64_check_update(_ptr(p_edge), _ptr(row_ptr), _ptr(coef), int(checks), int(edges),
                                        _ptr(out_msg), _stream(stream)), "cider_gf64_check_update")


def cider_amp_evidence(y, rows, slots: int, n_s: int, Q: int, rho: float, su2: float, iters: int, out_S,
                       stream=None) -> None:
    """Slot-wise AMP-MMSE evidence: y float32 [slots][n_s][2], rows int32
    [slots][n_s], out_S float32 [slots][Q], all device tensors."""
    check(lib().cider_amp_evidence(_ptr(y), _ptr(rows), int(slots), int(n_s), int(Q), float(rho), float(su2),
                                   int(iters), _ptr(out_S), _stream(stream)), "cider_amp_evidence")


def cider_evidence(y, sigma2: float, K: int, n: int, out_S=None, out_p=None, stream=None) -> None:
    check(lib().cider_evidence(_ptr(y), float(sigma2), K, n, _ptr(out_S), _ptr(out_p), _stream(stream)),
          "cider_evidence")


class Server:
    """Owns a cider_server (continuous batching of arriving bins on its own
    stream and worker thread); submit host buffers, poll or drain results."""

    def __init__(self, w: Weights, steps: int, opts: Optional[cider_opts] = None, max_slots: int = 64,
                 max_queue: int = 1 << 20, hbm_budget: int = 0, max_tokens: int = 1 << 18):
        cfg = cider_server_cfg()
        cfg.weights = w.handle
        cfg.opts = opts if opts is not None else cider_opts_default()
        cfg.steps, cfg.max_slots, cfg.max_queue = int(steps), int(max_slots), int(max_queue)
        cfg.hbm_budget, cfg.max_tokens = int(hbm_budget), int(max_tokens)
        self.cfg = cfg
        h = C.c_void_p()
        check(lib().cider_server_create(C.byref(cfg), C.byref(h)), "cider_server_create")
        self.handle = h
        self._keep = {}                 # request id -> host buffers the library reads or writes

    @staticmethod
    def budget_floor(w: Weights, steps: int, opts: Optional[cider_opts] = None, max_slots: int = 64) -> int:
        """Smallest hbm_budget a server of this model and slot count accepts."""
        cfg = cider_server_cfg()
        cfg.weights = w.handle
        cfg.opts = opts if opts is not None else cider_opts_default()
        cfg.steps, cfg.max_slots, cfg.max_queue, cfg.max_tokens = int(steps), int(max_slots), 1, 1
        out = C.c_size_t()
        check(lib().cider_server_budget_floor(C.byref(cfg), C.byref(out)), "cider_server_budget_floor")
        return int(out.value)

    def submit(self, y: np.ndarray, sigma2: float, code: Code, K: int, n: int) -> Tuple[int, np.ndarray]:
        """Queues a bin; returns (request id, host [K][n] uint8 array written when it is done)."""
        y = np.ascontiguousarray(y, dtype=np.float32)
        out = np.zeros((K, n), dtype=np.uint8)
        rid = C.c_uint64()
        check(lib().cider_server_submit(self.handle, y.ctypes.data, float(sigma2), code.handle, int(K), int(n),
                                        out.ctypes.data, C.byref(rid)), "cider_server_submit")
        self._keep[rid.value] = (y, out)
        return rid.value, out

    def poll(self, max_results: int = 4096) -> list:
        res = (cider_result * max_results)()
        got = C.c_int32()
        check(lib().cider_server_poll(self.handle, res, max_results, C.byref(got)), "cider_server_poll")
        done = [res[i] for i in range(got.value)]
        for r in done:
            self._keep.pop(r.id, None)
        return done

    def drain(self) -> None:
        check(lib().cider_server_drain(self.handle), "cider_server_drain")

    def close(self):
        if self.handle:
            lib().cider_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cider_profile_read(w: Weights, reset: bool = True) -> dict:
    """{kernel role: (launches, total ms)} from decodes run with opts.profile = 1."""
    arr = (cider_kernel_stat * 64)()
    n = C.c_int32()
    check(lib().cider_profile_read(w.handle, arr, 64, C.byref(n), int(reset)), "cider_profile_read")
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(n.value)}


def cider_tuning_read(w: Weights) -> list:
    """[(role, N, Kd, bucket, tile, best_ms, default_ms)] chosen by the autotuner
    (GEMM tile shapes; for the fused kernels' roles N = d, Kd = hidden width and
    tile = variant)."""
    arr = (cider_tuning_entry * 128)()
    n = C.c_int32()
    check(lib().cider_tuning_read(w.handle, arr, 128, C.byref(n)), "cider_tuning_read")
    return [(arr[i].role.decode(), arr[i].n, arr[i].kd, arr[i].bucket, arr[i].tile, arr[i].best_ms,
             arr[i].default_ms) for i in range(n.value)]


def cider_strerror(status: int) -> str:
    return lib().cider_strerror(status).decode()


def cider_last_error() -> str:
    return lib().cider_last_error().decode(errors="replace")
