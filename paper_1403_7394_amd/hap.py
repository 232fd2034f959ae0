"""ctypes binding of libhap (include/hap.h).

Argument marshalling only: every step of the method runs in the HIP library.
torch supplies device memory (tensors) and the stream (torch's current stream).
The library must have been built (``python -m paper_1403_7394_amd.build``);
``load()`` raises if it is missing, and nothing here falls back to another path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhap.so")

HAP_OK, HAP_E_ARG, HAP_E_DTYPE, HAP_E_OOM, HAP_E_HIP, HAP_E_STATE, HAP_E_UNSUPPORTED = range(7)
HAP_F32, HAP_F64 = 0, 1
BUILD_DIRECT, BUILD_GEMM, BUILD_BF16, BUILD_BF16X3, BUILD_DIRECT_L2 = 0, 1, 2, 3, 4
PREF_MEDIAN, PREF_SCALAR, PREF_VECTOR = 0, 1, 2
LAUNCH_STREAM = 2
LAUNCH_EAGER = 4
LAUNCH_UNFUSED = 8
LAUNCH_FUSED = 16   # reported by hap_get_launch: the MapReduce levels run in one fused pass
LAUNCH_BLOCKS = 32  # each workgroup takes a contiguous block of rows (default: rows interleaved)
PROBE_CACHED, PROBE_BLOCKS = 1, 2
SCHEDULE_SEQUENTIAL, SCHEDULE_MRHAP = 0, 1

# every symbol include/hap.h declares
EXPORTS = (
    "hap_version", "hap_status_string", "hap_last_error", "hap_build_similarity",
    "hap_median_offdiag", "hap_median_offdiag_noalloc", "hap_bandwidth_probe", "hap_workspace_size", "hap_init",
    "hap_iterate", "hap_exemplars",
    "hap_net_similarity", "hap_preference", "hap_read_messages", "hap_similarity_offsets", "hap_set_launch",
    "hap_set_points", "hap_set_row_count", "hap_get_row_count",
    "hap_get_launch", "hap_profile", "hap_profile_read", "hap_destroy",
    "hap_batch_workspace_size", "hap_batch_create", "hap_batch_run", "hap_batch_set_launch",
    "hap_batch_get_launch", "hap_batch_set_split", "hap_batch_get_split", "hap_batch_get_members", "hap_batch_destroy",
    "hap_warm_features", "hap_warm_targets", "hap_set_warm_start", "hap_set_warm_alpha", "hap_iterate_warm",
    "hap_iterate_warm_judged",
    "hap_mlp_param_count", "hap_mlp_workspace_size", "hap_mlp_forward", "hap_mlp_loss_grad", "hap_mlp_adam",
    "hap_mlp_train",
)
WARM_FEATURES = 32
HAP_BF16 = 2


class HapError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


class hap_params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("levels", ctypes.c_int32),
        ("damping", ctypes.c_double),
        ("pref_mode", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
        ("pref_scalar", ctypes.POINTER(ctypes.c_double)),
        ("pref_vec", ctypes.c_void_p),
        ("kappa", ctypes.c_double),
    ]


_lib = None

_c_i32p = ctypes.POINTER(ctypes.c_int32)
_c_dblp = ctypes.POINTER(ctypes.c_double)


def _declare(lib):
    V, I32, I64, U64, D, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t
    sig = {
        "hap_version": (ctypes.c_char_p, []),
        "hap_status_string": (ctypes.c_char_p, [I32]),
        "hap_last_error": (ctypes.c_char_p, []),
        "hap_build_similarity": (I32, [V, I64, I64, I64, I32, V, I64, I32, I32, D, U64, V]),
        "hap_median_offdiag": (I32, [V, I64, I64, I32, _c_dblp, V]),
        "hap_median_offdiag_noalloc": (I32, [V, I64, I64, I32, V, V]),
        "hap_bandwidth_probe": (I32, [I32, I32, ctypes.POINTER(V), ctypes.POINTER(V), I64, I64, I64, I64, I32, V]),
        "hap_workspace_size": (I32, [I64, I32, I32, ctypes.POINTER(SZ)]),
        "hap_init": (I32, [ctypes.POINTER(V), V, I64, I64, I32, ctypes.POINTER(hap_params), V, SZ, V]),
        "hap_iterate": (I32, [V, I32, I32, _c_i32p, _c_i32p]),
        "hap_exemplars": (I32, [V, I32, V, _c_i32p]),
        "hap_net_similarity": (I32, [V, I32, V, I64, I64, I32, _c_dblp]),
        "hap_preference": (I32, [V, _c_dblp]),
        "hap_read_messages": (I32, [V, I32, V, V, I64, V, V, V]),
        "hap_set_launch": (I32, [V, I32, I32, I32, I32]),
        "hap_set_points": (I32, [V, V, I64, I64, I64, I32]),
        "hap_set_row_count": (I32, [V, I64]),
        "hap_get_row_count": (I32, [V, ctypes.POINTER(I64)]),
        "hap_get_launch": (I32, [V, _c_i32p, _c_i32p, _c_i32p, _c_i32p]),
        "hap_profile": (I32, [V, I32]),
        "hap_profile_read": (I32, [V, _c_dblp, ctypes.POINTER(I64), _c_dblp, ctypes.POINTER(I64)]),
        "hap_destroy": (I32, [V]),
        "hap_batch_workspace_size": (I32, [I32, _c_i32p, I64, I32, ctypes.POINTER(SZ)]),
        "hap_batch_create": (I32, [ctypes.POINTER(V), I32, _c_i32p, I64, I32, V, SZ, V]),
        "hap_batch_run": (I32, [V, V, D, I32, I32, V, V, V, V]),
        "hap_batch_set_launch": (I32, [V, I32, I32, I32]),
        "hap_batch_get_launch": (I32, [V, _c_i32p, _c_i32p, _c_i32p]),
        "hap_batch_set_split": (I32, [V, I32, I32, V]),
        "hap_batch_get_split": (I32, [V, _c_i32p, _c_i32p]),
        "hap_batch_get_members": (I32, [V, _c_i32p, _c_i32p]),
        "hap_batch_destroy": (I32, [V]),
        "hap_similarity_offsets": (I32, [V, I32, V]),
        "hap_warm_features": (I32, [V, V, I64]),
        "hap_warm_targets": (I32, [V, V, I64]),
        "hap_set_warm_start": (I32, [V, V, I64]),
        "hap_set_warm_alpha": (I32, [V, V, I64]),
        "hap_iterate_warm": (I32, [V, V, I64, I32, I32, _c_i32p, _c_i32p, _c_i32p]),
        "hap_iterate_warm_judged": (I32, [V, V, I64, I32, I32, V, I64, I64, I32, _c_i32p, _c_i32p, _c_i32p,
                                          _c_dblp, _c_dblp]),
        "hap_mlp_param_count": (I64, [I32, I32, I32]),
        "hap_mlp_workspace_size": (I32, [I32, I32, I32, I64, ctypes.POINTER(SZ)]),
        "hap_mlp_forward": (I32, [V, I32, I32, I32, I32, V, I64, I64, V, I64, V, SZ, V]),
        "hap_mlp_loss_grad": (I32, [V, I32, I32, I32, I32, V, I64, V, I64, I64, V, V, V, SZ, V]),
        "hap_mlp_adam": (I32, [V, V, V, I64, I64, D, D, D, D, V]),
        "hap_mlp_train": (I32, [V, V, I32, I32, I32, I32, I64, V, I64, V, I64, I64, V, I64, I64, D, V, V, SZ, V]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args


def load(path: str | None = None):
    """Load libhap.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libhap not built: {p} is missing (run python -m paper_1403_7394_amd.build)")
    lib = ctypes.CDLL(p)
    _declare(lib)
    _lib = lib
    return lib


def _check(fn, status):
    if status != HAP_OK:
        msg = _lib.hap_last_error().decode(errors="replace")
        raise HapError(fn, status, msg)


def _dtype_code(t):
    import torch
    if t.dtype == torch.float32:
        return HAP_F32
    if t.dtype == torch.float64:
        return HAP_F64
    raise TypeError(f"unsupported dtype {t.dtype}")


def _stream(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ld(t):
    """Leading dimension (elements) of a row-major 2-D tensor view."""
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("expected a row-major 2-D tensor")
    return t.stride(0)


def version() -> str:
    return load().hap_version().decode()


def build_similarity(X, S, mode: int = BUILD_DIRECT, noise_rel: float = 0.0, seed: int = 0, stream=None):
    """S[:n, :n] <- -||x_i - x_j||^2 (see hap_build_similarity)."""
    lib = load()
    n, d = X.shape
    _check("hap_build_similarity", lib.hap_build_similarity(
        ctypes.c_void_p(X.data_ptr()), n, d, _ld(X), _dtype_code(X), ctypes.c_void_p(S.data_ptr()), _ld(S),
        _dtype_code(S), mode, float(noise_rel), ctypes.c_uint64(seed & ((1 << 64) - 1)), _stream(stream)))
    return S


def median_offdiag(S, stream=None) -> float:
    lib = load()
    out = ctypes.c_double()
    _check("hap_median_offdiag", lib.hap_median_offdiag(
        ctypes.c_void_p(S.data_ptr()), S.shape[0], _ld(S), _dtype_code(S), ctypes.byref(out), _stream(stream)))
    return out.value


def median_offdiag_noalloc(S, out, stream=None) -> None:
    """hap_median_offdiag_noalloc: the median into `out` (a float64 device tensor of one element),
    enqueued on the stream without any allocation or synchronisation."""
    lib = load()
    _check("hap_median_offdiag_noalloc", lib.hap_median_offdiag_noalloc(
        ctypes.c_void_p(S.data_ptr()), S.shape[0], _ld(S), _dtype_code(S), ctypes.c_void_p(out.data_ptr()),
        _stream(stream)))


def bandwidth_probe(inputs, outputs, sink=None, rows_per_block: int = 32, stream=None, cached: bool = False,
                    blocks: bool = False) -> None:
    """hap_bandwidth_probe: reads the 2-D FP32 device tensors `inputs` and writes `outputs`, all
    of one shape and row stride (no inputs: the pure-write mix).  With no outputs (the pure-read
    mix) `sink` is a one-element FP32 device tensor the kernel may store to.  cached / blocks:
    HAP_PROBE_CACHED / HAP_PROBE_BLOCKS."""
    import torch
    lib = load()
    first = inputs[0] if inputs else outputs[0]
    rows, cols = first.shape
    ld = _ld(first)
    for t in list(inputs) + list(outputs):
        if t.dtype != torch.float32 or tuple(t.shape) != (rows, cols) or _ld(t) != ld or not t.is_cuda:
            raise ValueError("bandwidth_probe: every array must be an FP32 device tensor of the same shape and stride")
    if not outputs and (sink is None or sink.dtype != torch.float32 or sink.numel() < 1 or not sink.is_cuda):
        raise ValueError("bandwidth_probe: the pure-read mix needs a one-element FP32 device sink")
    ins = (ctypes.c_void_p * 3)(*[ctypes.c_void_p(t.data_ptr()) for t in inputs]) if inputs else None
    targets = list(outputs) if outputs else [sink]
    outs = (ctypes.c_void_p * 2)(*[ctypes.c_void_p(t.data_ptr()) for t in targets])
    flags = (PROBE_CACHED if cached else 0) | (PROBE_BLOCKS if blocks else 0)
    _check("hap_bandwidth_probe", lib.hap_bandwidth_probe(len(inputs), len(outputs), ins, outs, rows, cols,
                                                          ld, rows_per_block, flags, _stream(stream)))


def workspace_size(n: int, levels: int, dtype_code: int) -> int:
    lib = load()
    b = ctypes.c_size_t()
    _check("hap_workspace_size", lib.hap_workspace_size(n, levels, dtype_code, ctypes.byref(b)))
    return b.value


@dataclass
class IterResult:
    iters: int
    converged: bool


class Hap:
    """One HAP problem on the GPU (wraps a hap_ctx).  S must outlive this object."""

    def __init__(self, S, levels: int, damping: float, pref=None, workspace=None, stream=None,
                 schedule: int = SCHEDULE_SEQUENTIAL, kappa: float = 0.0):
        import torch
        lib = load()
        self._lib = lib
        self.S = S                      # keep the borrowed similarity alive
        self.n = S.shape[0]
        self.levels = levels
        self.dtype = S.dtype
        self._stream_obj = stream if stream is not None else torch.cuda.current_stream()
        p = hap_params()
        p.struct_size = ctypes.sizeof(hap_params)
        p.levels = levels
        p.damping = float(damping)
        p.schedule = int(schedule)
        p.kappa = float(kappa)
        self.schedule = int(schedule)
        self.kappa = float(kappa)
        self._pref_keep = None
        if pref is None:
            p.pref_mode = PREF_MEDIAN
        elif isinstance(pref, torch.Tensor):
            if pref.dim() == 1:
                pref = pref.reshape(1, -1).expand(levels, -1)
            pref = pref.to(device=S.device, dtype=S.dtype).contiguous()
            self._pref_keep = pref
            p.pref_mode = PREF_VECTOR
            p.pref_vec = ctypes.c_void_p(pref.data_ptr())
        else:
            vals = [float(pref)] * levels if not hasattr(pref, "__len__") else [float(v) for v in pref]
            arr = (ctypes.c_double * levels)(*vals)
            self._pref_keep = arr
            p.pref_mode = PREF_SCALAR
            p.pref_scalar = ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))
        ws_ptr, ws_bytes = None, 0
        if workspace is not None:
            ws_ptr, ws_bytes = ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()
            self._ws_keep = workspace
        ctx = ctypes.c_void_p()
        _check("hap_init", lib.hap_init(ctypes.byref(ctx), ctypes.c_void_p(S.data_ptr()), self.n, _ld(S),
                                        _dtype_code(S), ctypes.byref(p), ws_ptr, ws_bytes,
                                        ctypes.c_void_p(self._stream_obj.cuda_stream)))
        self._ctx = ctx

    def close(self):
        if getattr(self, "_ctx", None):
            _check("hap_destroy", self._lib.hap_destroy(self._ctx))
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def iterate(self, max_iters: int, stable_iters: int = 0) -> IterResult:
        it, cv = ctypes.c_int32(), ctypes.c_int32()
        _check("hap_iterate", self._lib.hap_iterate(self._ctx, max_iters, stable_iters, ctypes.byref(it), ctypes.byref(cv)))
        return IterResult(it.value, bool(cv.value))

    def exemplars(self, level: int, out=None):
        """(labels tensor int32 [n] on the device, number of distinct exemplars)."""
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=torch.int32, device=self.S.device)
        k = ctypes.c_int32()
        _check("hap_exemplars", self._lib.hap_exemplars(self._ctx, level, ctypes.c_void_p(out.data_ptr()), ctypes.byref(k)))
        return out, k.value

    def labels(self):
        import torch
        return torch.stack([self.exemplars(l)[0] for l in range(self.levels)])

    def net_similarity(self, level: int = -1, X=None) -> float:
        out = ctypes.c_double()
        if X is None:
            st = self._lib.hap_net_similarity(self._ctx, level, None, 0, 0, 0, ctypes.byref(out))
        else:
            st = self._lib.hap_net_similarity(self._ctx, level, ctypes.c_void_p(X.data_ptr()), X.shape[1], _ld(X),
                                              _dtype_code(X), ctypes.byref(out))
        _check("hap_net_similarity", st)
        return out.value

    def preference(self):
        arr = (ctypes.c_double * self.levels)()
        _check("hap_preference", self._lib.hap_preference(self._ctx, arr))
        return list(arr)

    def messages(self, level: int):
        """dict of rho, alpha (n x n) and c, phi, tau (n) of `level` after the last sweep."""
        import torch
        dev = self.S.device
        rho = torch.empty(self.n, self.n, dtype=self.dtype, device=dev)
        alpha = torch.empty_like(rho)
        c = torch.empty(self.n, dtype=self.dtype, device=dev)
        phi = torch.empty_like(c)
        tau = torch.empty_like(c)
        P = lambda t: ctypes.c_void_p(t.data_ptr())
        _check("hap_read_messages", self._lib.hap_read_messages(self._ctx, level, P(rho), P(alpha), self.n, P(c), P(phi), P(tau)))
        return dict(rho=rho, alpha=alpha, c=c, phi=phi, tau=tau)

    def offsets(self, level: int):
        """Eq. 2.7 row offsets delta^l (n) of `level` after the last sweep (0 when kappa = 0)."""
        import torch
        d = torch.empty(self.n, dtype=self.dtype, device=self.S.device)
        _check("hap_similarity_offsets", self._lib.hap_similarity_offsets(self._ctx, level, ctypes.c_void_p(d.data_ptr())))
        return d

    def set_launch(self, threads=0, chunks=0, rows_per_block=0, streaming=None, eager=None, unfused=None,
                   blocks=None):
        """Launch shape; streaming / eager / unfused / blocks None keep the current choice (the
        flags are set together)."""
        if streaming is None and eager is None and unfused is None and blocks is None:
            flags = -1
        else:
            cur = self.launch_flags()
            st = bool(cur & LAUNCH_STREAM) if streaming is None else streaming
            ea = bool(cur & LAUNCH_EAGER) if eager is None else eager
            uf = bool(cur & LAUNCH_UNFUSED) if unfused is None else unfused
            bl = bool(cur & LAUNCH_BLOCKS) if blocks is None else blocks
            flags = ((LAUNCH_STREAM if st else 0) | (LAUNCH_EAGER if ea else 0) | (LAUNCH_UNFUSED if uf else 0)
                     | (LAUNCH_BLOCKS if bl else 0))
        _check("hap_set_launch", self._lib.hap_set_launch(self._ctx, threads, chunks, rows_per_block, flags))

    def launch_flags(self) -> int:
        """The HAP_LAUNCH_* bits in effect."""
        a, b, c, f = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check("hap_get_launch", self._lib.hap_get_launch(self._ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                                          ctypes.byref(f)))
        return f.value

    def set_row_count(self, rows: int):
        """Update rows [0, rows) only: one block of a run split by rows (n: the whole problem)."""
        _check("hap_set_row_count", self._lib.hap_set_row_count(self._ctx, int(rows)))

    def get_row_count(self) -> int:
        r = ctypes.c_int64()
        _check("hap_get_row_count", self._lib.hap_get_row_count(self._ctx, ctypes.byref(r)))
        return r.value

    def set_points(self, X=None):
        """Points mode: the row pass recomputes s_ij from X (the FP32 points S was built from
        with BUILD_DIRECT, no noise) instead of reading S.  None switches it off.  The library
        refuses points whose count differs from n or whose sampled distances differ from S."""
        if X is None:
            _check("hap_set_points", self._lib.hap_set_points(self._ctx, None, 0, 0, 0, 0))
            self._points_keep = None
            return
        _check("hap_set_points", self._lib.hap_set_points(self._ctx, ctypes.c_void_p(X.data_ptr()), X.shape[0],
                                                          X.shape[1], _ld(X), _dtype_code(X)))
        self._points_keep = X

    def profile(self, enable, every: int = 1):
        """Per-launch event timing of every `every`-th sweep (enable False stops)."""
        _check("hap_profile", self._lib.hap_profile(self._ctx, int(every) if enable else 0))

    def profile_read(self):
        """(row pass ms, row pass launches, column-sum ms, column-sum launches)."""
        a, b, c, d = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
        _check("hap_profile_read", self._lib.hap_profile_read(self._ctx, ctypes.byref(a), ctypes.byref(b),
                                                              ctypes.byref(c), ctypes.byref(d)))
        return a.value, b.value, c.value, d.value

    # ---------------------------------------------------------------- warm start
    def warm_features(self, out=None):
        """(n, WARM_FEATURES) FP32 features of every point (hap_warm_features)."""
        import torch
        if out is None:
            out = torch.empty(self.n, WARM_FEATURES, dtype=torch.float32, device=self.S.device)
        _check("hap_warm_features", self._lib.hap_warm_features(self._ctx, ctypes.c_void_p(out.data_ptr()), _ld(out)))
        return out

    def warm_targets(self, out=None):
        """(n, levels) FP32 training targets of the current state (hap_warm_targets)."""
        import torch
        if out is None:
            out = torch.empty(self.n, self.levels, dtype=torch.float32, device=self.S.device)
        _check("hap_warm_targets", self._lib.hap_warm_targets(self._ctx, ctypes.c_void_p(out.data_ptr()), _ld(out)))
        return out

    def set_warm_start(self, Y=None):
        """Restart from the warm availabilities of network outputs Y (n, levels), or cold."""
        ptr, ld = (None, 0) if Y is None else (ctypes.c_void_p(Y.data_ptr()), _ld(Y))
        self._warm_keep = Y
        _check("hap_set_warm_start", self._lib.hap_set_warm_start(self._ctx, ptr, ld))

    def set_warm_alpha(self, alpha_diag0):
        """Restart from given initial availabilities: alpha_diag0 (n, levels), device, the
        working type; alpha^l_jj = alpha_diag0[j, l], alpha^l_ij = min(0, alpha_diag0[j, l])."""
        import torch
        if alpha_diag0 is None or not alpha_diag0.is_cuda or alpha_diag0.dtype != self.dtype or \
                alpha_diag0.dim() != 2 or alpha_diag0.shape[0] != self.n or alpha_diag0.stride(1) != 1:
            raise ValueError("set_warm_alpha: a device (n, levels) tensor of the working type, unit column stride")
        self._warm_keep = alpha_diag0
        _check("hap_set_warm_alpha", self._lib.hap_set_warm_alpha(self._ctx, ctypes.c_void_p(alpha_diag0.data_ptr()),
                                                                  alpha_diag0.stride(0)))

    def iterate_warm(self, Y, max_iters: int, stable_iters: int):
        """Warm run with the cold start as fallback: (IterResult, fell_back)."""
        ptr, ld = (None, 0) if Y is None else (ctypes.c_void_p(Y.data_ptr()), _ld(Y))
        it, cv, fb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check("hap_iterate_warm", self._lib.hap_iterate_warm(self._ctx, ptr, ld, max_iters, stable_iters,
                                                              ctypes.byref(it), ctypes.byref(cv), ctypes.byref(fb)))
        return IterResult(it.value, bool(cv.value)), bool(fb.value)

    def iterate_warm_judged(self, Y, max_iters: int, stable_iters: int, X=None):
        """Warm run judged by the cold start: both run, the one with the larger net similarity
        summed over levels (from X in FP64 when given, else from S; the warm run on a tie) is
        kept, converged or not.  Returns (IterResult, fell_back, ns_warm, ns_cold)."""
        if Y is None:
            raise ValueError("iterate_warm_judged needs a warm start Y")
        it, cv, fb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        nw, nc = ctypes.c_double(), ctypes.c_double()
        if X is None:
            xp, d, ldx, xdt = None, 0, 0, 0
        else:
            if X.dim() != 2 or X.shape[0] != self.n or X.device != self.S.device:
                raise ValueError("X must be (n, d) on the context's device")
            xp, d, ldx, xdt = ctypes.c_void_p(X.data_ptr()), X.shape[1], _ld(X), _dtype_code(X)
        _check("hap_iterate_warm_judged", self._lib.hap_iterate_warm_judged(
            self._ctx, ctypes.c_void_p(Y.data_ptr()), _ld(Y), max_iters, stable_iters, xp, d, ldx, xdt,
            ctypes.byref(it), ctypes.byref(cv), ctypes.byref(fb), ctypes.byref(nw), ctypes.byref(nc)))
        return IterResult(it.value, bool(cv.value)), bool(fb.value), nw.value, nc.value

    def get_launch(self):
        """(threads, chunks, rows_per_block, streaming)."""
        a, b, c, f = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check("hap_get_launch", self._lib.hap_get_launch(self._ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                                          ctypes.byref(f)))
        return a.value, b.value, c.value, bool(f.value & LAUNCH_STREAM)


class HapBatch:
    """Many independent FP32 problems (2..2048 points each) run by one persistent launch.

    sizes: list of point counts; X (run()): device FP32 tensor (sum(sizes), d), the problems'
    points stacked in order.
    """

    def __init__(self, sizes, d: int, levels: int, workspace=None, stream=None):
        import torch
        lib = load()
        self._lib = lib
        self.sizes = [int(v) for v in sizes]
        self.count = len(self.sizes)
        self.d = int(d)
        self.levels = int(levels)
        self.offsets = [0]
        for v in self.sizes:
            self.offsets.append(self.offsets[-1] + v)
        arr = (ctypes.c_int32 * self.count)(*self.sizes)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        ws_ptr, ws_bytes = None, 0
        if workspace is not None:
            ws_ptr, ws_bytes = ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()
            self._ws_keep = workspace
        h = ctypes.c_void_p()
        _check("hap_batch_create", lib.hap_batch_create(ctypes.byref(h), self.count, arr, self.d, self.levels,
                                                        ws_ptr, ws_bytes, ctypes.c_void_p(self._stream.cuda_stream)))
        self._h = h

    @staticmethod
    def workspace_size(sizes, d, levels) -> int:
        lib = load()
        arr = (ctypes.c_int32 * len(sizes))(*[int(v) for v in sizes])
        b = ctypes.c_size_t()
        _check("hap_batch_workspace_size", lib.hap_batch_workspace_size(len(sizes), arr, d, levels, ctypes.byref(b)))
        return b.value

    def outputs(self, device):
        """Fresh output tensors: labels, net similarity, iterations."""
        import torch
        labels = torch.empty(self.levels * self.offsets[-1], dtype=torch.int32, device=device)
        ns = torch.empty((self.count, self.levels + 1), dtype=torch.float64, device=device)
        iters = torch.empty(self.count, dtype=torch.int32, device=device)
        return labels, ns, iters

    def run(self, X, damping, max_iters, stable_iters=0, out=None, stream=None):
        import torch
        labels, ns, iters = out if out is not None else self.outputs(X.device)
        st = stream if stream is not None else torch.cuda.current_stream()
        P = lambda t: ctypes.c_void_p(t.data_ptr())
        _check("hap_batch_run", self._lib.hap_batch_run(self._h, P(X), float(damping), int(max_iters), int(stable_iters),
                                                        P(labels), P(ns), P(iters), ctypes.c_void_p(st.cuda_stream)))
        return labels, ns, iters

    def labels_of(self, labels, b):
        """(levels, n_b) view of problem b's labels."""
        o, n = self.offsets[b], self.sizes[b]
        return labels[self.levels * o: self.levels * (o + n)].view(self.levels, n)

    def set_launch(self, threads=0, workgroups=0, row_groups=0):
        _check("hap_batch_set_launch", self._lib.hap_batch_set_launch(self._h, threads, workgroups, row_groups))

    def get_launch(self):
        """(threads, workgroups, row_groups)"""
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check("hap_batch_get_launch", self._lib.hap_batch_get_launch(self._h, ctypes.byref(a), ctypes.byref(b),
                                                                      ctypes.byref(c)))
        return a.value, b.value, c.value

    def set_split(self, split_n: int, max_members: int = 4):
        """Share problems of more than split_n points among gangs of up to max_members
        workgroups (split_n = 0: no split)."""
        _check("hap_batch_set_split", self._lib.hap_batch_set_split(self._h, int(split_n), int(max_members),
                                                                      ctypes.c_void_p(self._stream.cuda_stream)))

    def get_split(self):
        """(split_n, max_members)"""
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check("hap_batch_get_split", self._lib.hap_batch_get_split(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def members(self):
        """(members, rows per member) of every problem under the current split."""
        k = (ctypes.c_int32 * self.count)()
        r = (ctypes.c_int32 * self.count)()
        _check("hap_batch_get_members", self._lib.hap_batch_get_members(self._h, k, r))
        return list(k), list(r)

    def close(self):
        if getattr(self, "_h", None):
            _check("hap_batch_destroy", self._lib.hap_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """The warm start's perceptron (n_in -> hidden -> hidden -> n_out, ReLU) on the GPU.

    params: flat FP32 device tensor (hap_mlp_param_count values); precision HAP_F32 or
    HAP_BF16 (operands of every product rounded to BF16, FP32 accumulation)."""

    def __init__(self, params, n_in: int, hidden: int, n_out: int, precision: int = HAP_BF16, stream=None):
        import torch
        self._lib = load()
        self.n_in, self.hidden, self.n_out, self.precision = n_in, hidden, n_out, precision
        cnt = self._lib.hap_mlp_param_count(n_in, hidden, n_out)
        if cnt < 0 or params.numel() != cnt or params.dtype != torch.float32 or not params.is_contiguous():
            raise ValueError("params must be a contiguous FP32 tensor of hap_mlp_param_count values")
        self.params = params
        self.count = cnt
        self.opt_state = torch.zeros(2 * cnt, dtype=torch.float32, device=params.device)
        self.step = 0
        self._stream_obj = stream
        self._ws = None

    def _workspace(self, rows: int):
        import torch
        b = ctypes.c_size_t()
        _check("hap_mlp_workspace_size", self._lib.hap_mlp_workspace_size(self.n_in, self.hidden, self.n_out, rows,
                                                                            ctypes.byref(b)))
        if self._ws is None or self._ws.numel() < b.value:
            self._ws = torch.empty(b.value, dtype=torch.uint8, device=self.params.device)
        return ctypes.c_void_p(self._ws.data_ptr()), self._ws.numel()

    def forward(self, X, out=None):
        import torch
        rows = X.shape[0]
        if out is None:
            out = torch.empty(rows, self.n_out, dtype=torch.float32, device=X.device)
        ws, nb = self._workspace(rows)
        P = lambda t: ctypes.c_void_p(t.data_ptr())
        _check("hap_mlp_forward", self._lib.hap_mlp_forward(P(self.params), self.n_in, self.hidden, self.n_out,
                                                            self.precision, P(X), _ld(X), rows, P(out), _ld(out), ws,
                                                            nb, _stream(self._stream_obj)))
        return out

    def loss_grad(self, X, T):
        """(loss tensor (device double, shape []), gradient (flat FP32, like params))."""
        import torch
        rows = X.shape[0]
        grad = torch.empty_like(self.params)
        loss = torch.empty((), dtype=torch.float64, device=X.device)
        ws, nb = self._workspace(rows)
        P = lambda t: ctypes.c_void_p(t.data_ptr())
        _check("hap_mlp_loss_grad", self._lib.hap_mlp_loss_grad(P(self.params), self.n_in, self.hidden, self.n_out,
                                                                self.precision, P(X), _ld(X), P(T), _ld(T), rows,
                                                                P(grad), P(loss), ws, nb, _stream(self._stream_obj)))
        return loss, grad

    def adam(self, grad, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.step += 1
        P = lambda t: ctypes.c_void_p(t.data_ptr())
        _check("hap_mlp_adam", self._lib.hap_mlp_adam(P(self.params), P(grad), P(self.opt_state), self.count, self.step,
                                                      lr, beta1, beta2, eps, _stream(self._stream_obj)))

    def train(self, X, T, idx, batch: int, steps: int, lr: float, loss_hist=None):
        """Minibatch Adam over rows idx (device int32, batch*steps entries); returns the
        per-step losses (device double tensor)."""
        import torch
        if idx.dtype != torch.int32 or idx.numel() < batch * steps:
            raise ValueError("idx must be int32 with batch*steps entries")
        if loss_hist is None:
            loss_hist = torch.empty(steps, dtype=torch.float64, device=X.device)
        ws, nb = self._workspace(batch)
        P = lambda t: ctypes.c_void_p(t.data_ptr())
        _check("hap_mlp_train", self._lib.hap_mlp_train(P(self.params), P(self.opt_state), self.n_in, self.hidden,
                                                        self.n_out, self.precision, self.step, P(X), _ld(X), P(T),
                                                        _ld(T), X.shape[0], P(idx), batch, steps, lr, P(loss_hist),
                                                        ws, nb, _stream(self._stream_obj)))
        self.step += steps
        return loss_hist
