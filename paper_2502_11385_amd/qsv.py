"""ctypes binding of libqsv.so (argument marshalling only).

Every call maps one-to-one onto the C ABI declared in ``include/qsv.h``; all
arithmetic runs in the HIP library.  PyTorch is used only for device
buffers and streams.  If the library has not been built this module raises
at import: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Iterable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqsv.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first "
        "(python -m paper_2502_11385_amd.build)")

# PyTorch ships its own HIP runtime.  Importing it first makes libqsv bind
# to that same runtime (same soname) instead of mapping a second one, so that
# tensors, streams and the library share one device context.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

QSV_OK = 0
QSV_ERR_INVALID_ARG = 1
QSV_ERR_OUT_OF_MEMORY = 2
QSV_ERR_DEVICE = 3
QSV_ERR_UNSUPPORTED = 4
QSV_ERR_BUDGET = 5
QSV_ERR_CANCELLED = 6
QSV_ERR_TIMEOUT = 7
QSV_C64 = 1
QSV_C128 = 2
PLAN_AUTO, PLAN_PLAIN, PLAN_TILED, PLAN_FUSED = 0, 1, 2, 3
MAX_QUBITS = 34

EXPORTED = [
    "qsv_alloc", "qsv_wrap", "qsv_free", "qsv_init_basis", "qsv_apply_gate",
    "qsv_apply_fused", "qsv_apply_fused_outputs", "qsv_last_plan_stats",
    "qsv_plan_describe",
    "qsv_gate_matrix", "qsv_probabilities", "qsv_norm", "qsv_renormalize",
    "qsv_marginal", "qsv_sample", "qsv_get_amplitudes", "qsv_set_amplitudes",
    "qsv_info", "qsv_sync", "qsv_last_error", "qsv_version",
    "qsv_set_profiling", "qsv_pass_times", "qsv_autotune_fused",
    "qsv_renormalize_noalloc",
    "qsv_batch_create", "qsv_batch_out_offsets", "qsv_batch_launch",
    "qsv_batch_stats", "qsv_batch_free", "qsv_gate_matrices",
    "qsv_server_create", "qsv_server_submit", "qsv_server_wait",
    "qsv_server_release", "qsv_server_stats", "qsv_server_destroy",
    "qsv_server_wait_timeout", "qsv_server_cancel", "qsv_debug_inject",
    "qsv_clock", "qsv_debug_emulate_tiled", "qsv_plan_program_stats",
    "qsv_cut_workspace_bytes", "qsv_cut_reconstruct",
    "qsv_top_k", "qsv_expectation_pauli", "qsv_permute_qubits",
]


class QsvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"qsv status {status}: {msg}")
        self.status = status


class qsv_circuit(C.Structure):
    _fields_ = [("n_gates", C.c_size_t),
                ("k", C.POINTER(C.c_int32)),
                ("c", C.POINTER(C.c_int32)),
                ("qubits", C.POINTER(C.c_int32)),
                ("matrices", C.POINTER(C.c_double))]


class qsv_fuse_opts(C.Structure):
    _fields_ = [("strategy", C.c_int32), ("tile_log2", C.c_int32),
                ("k_max", C.c_int32), ("low_qubits", C.c_int32),
                ("reg_log2", C.c_int32)]


class qsv_variant(C.Structure):
    _fields_ = [("width", C.c_int32), ("body", qsv_circuit),
                ("n_inputs", C.c_int32),
                ("input_qubits", C.POINTER(C.c_int32)),
                ("input_labels", C.POINTER(C.c_int32)),
                ("n_outputs", C.c_int32),
                ("output_qubits", C.POINTER(C.c_int32)),
                ("output_bases", C.POINTER(C.c_int32))]


class qsv_outputs(C.Structure):
    _fields_ = [("probs_dev", C.c_void_p), ("probs_fp64", C.c_int32),
                ("marg_m", C.c_int32),
                ("marg_qubits", C.POINTER(C.c_int32)),
                ("marg_out", C.POINTER(C.c_double)),
                ("n_shots", C.c_uint64), ("shot_seed", C.c_uint64),
                ("shots_out", C.POINTER(C.c_uint64))]


class qsv_batch_opts(C.Structure):
    _fields_ = [("tile_log2", C.c_int32), ("reg_log2", C.c_int32),
                ("grid", C.c_int32), ("autotune", C.c_int32),
                ("use_graph", C.c_int32), ("out_fp64", C.c_int32)]


class qsv_server_opts(C.Structure):
    _fields_ = [("budget_bytes", C.c_uint64), ("max_batch", C.c_int32),
                ("small_width", C.c_int32), ("n_streams", C.c_int32),
                ("serial", C.c_int32)]


class qsv_request(C.Structure):
    _fields_ = [("width", C.c_int32), ("prec", C.c_int32),
                ("body", qsv_circuit), ("want_samples", C.c_int32),
                ("shots", C.c_uint64), ("seed", C.c_uint64)]


class qsv_cut_spec(C.Structure):
    _fields_ = [("n_sub", C.c_int32), ("n_cuts", C.c_int32),
                ("n_qubits", C.c_int32),
                ("widths", C.POINTER(C.c_int32)),
                ("out_qubit", C.POINTER(C.c_int32)),
                ("cut_in", C.POINTER(C.c_int32)),
                ("cut_out", C.POINTER(C.c_int32))]


class qsv_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("width", C.c_int32),
                ("prec", C.c_int32), ("is_samples", C.c_int32),
                ("batched", C.c_int32), ("pad", C.c_int32),
                ("n_out", C.c_uint64), ("data", C.c_void_p),
                ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_start", C.c_double), ("t_done", C.c_double)]


_p = C.c_void_p
_i32 = C.c_int32
_u64 = C.c_uint64
_pi32 = C.POINTER(C.c_int32)
_pd = C.POINTER(C.c_double)
_pu64 = C.POINTER(C.c_uint64)

_SIGS = {
    "qsv_alloc": [_i32, _i32, _p, C.POINTER(_p)],
    "qsv_wrap": [_i32, _i32, _p, C.c_size_t, _p, C.POINTER(_p)],
    "qsv_free": [_p],
    "qsv_init_basis": [_p, _u64],
    "qsv_apply_gate": [_p, _pi32, _i32, _pi32, _i32, _pd],
    "qsv_apply_fused": [_p, C.POINTER(qsv_circuit), C.POINTER(qsv_fuse_opts)],
    "qsv_apply_fused_outputs": [_p, C.POINTER(qsv_circuit),
                                C.POINTER(qsv_fuse_opts),
                                C.POINTER(qsv_outputs)],
    "qsv_last_plan_stats": [_p, _pu64, _i32],
    "qsv_plan_describe": [C.POINTER(qsv_circuit), _i32, _i32,
                          C.POINTER(qsv_fuse_opts), _pi32, _pi32, _pi32,
                          _pu64, _pi32],
    "qsv_gate_matrix": [C.c_char_p, _pd, _i32, _pd, _pi32],
    "qsv_gate_matrices": [C.c_char_p, _pd, _i32, C.c_size_t, _pd],
    "qsv_debug_emulate_tiled": [C.POINTER(qsv_circuit), _i32,
                                C.POINTER(qsv_fuse_opts), _pd],
    "qsv_plan_program_stats": [C.POINTER(qsv_circuit), _i32, _i32,
                               C.POINTER(qsv_fuse_opts), _pu64, _i32],
    "qsv_probabilities": [_p, _p, _i32],
    "qsv_norm": [_p, _pd],
    "qsv_renormalize": [_p, _pd],
    "qsv_renormalize_noalloc": [_p, _pd],
    "qsv_marginal": [_p, _pi32, _i32, _pd],
    "qsv_sample": [_p, _u64, _u64, _pu64],
    "qsv_get_amplitudes": [_p, _p],
    "qsv_set_amplitudes": [_p, _p],
    "qsv_info": [_p, C.POINTER(_p), _pi32, _pi32],
    "qsv_sync": [_p],
    "qsv_set_profiling": [_p, _i32],
    "qsv_batch_create": [C.POINTER(qsv_variant), C.c_size_t, _i32,
                         C.POINTER(qsv_batch_opts), _p, C.POINTER(_p)],
    "qsv_batch_out_offsets": [_p, _pu64],
    "qsv_batch_launch": [_p, _p],
    "qsv_batch_stats": [_p, _pu64, _i32],
    "qsv_batch_free": [_p],
    "qsv_server_create": [C.POINTER(qsv_server_opts), C.POINTER(_p)],
    "qsv_server_submit": [_p, C.POINTER(qsv_request), _pu64],
    "qsv_server_wait": [_p, _u64, C.POINTER(qsv_result)],
    "qsv_server_wait_timeout": [_p, _u64, C.c_double, C.POINTER(qsv_result)],
    "qsv_server_cancel": [_p, _u64],
    "qsv_debug_inject": [_i32, _i32],
    "qsv_server_release": [_p, _u64],
    "qsv_server_stats": [_p, _pu64, _i32],
    "qsv_server_destroy": [_p],
    "qsv_pass_times": [_p, C.POINTER(C.c_float), _pi32, _i32, _pi32],
    "qsv_autotune_fused": [_p, C.POINTER(qsv_circuit), C.POINTER(qsv_fuse_opts),
                           _i32, C.POINTER(qsv_fuse_opts),
                           C.POINTER(C.c_float), C.POINTER(C.c_float), _pi32],
    "qsv_top_k": [_p, C.c_uint32, _pu64, _pd],
    "qsv_permute_qubits": [_p, _pi32],
    "qsv_expectation_pauli": [_p, _i32, _pu64, _pu64, _pd],
    "qsv_cut_workspace_bytes": [C.POINTER(qsv_cut_spec), _pu64],
    "qsv_cut_reconstruct": [C.POINTER(qsv_cut_spec), _p, _i32, _u64, _pu64,
                            _p, _u64, _p, _p],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
_lib.qsv_last_error.restype = C.c_char_p
_lib.qsv_last_error.argtypes = []
_lib.qsv_version.restype = C.c_char_p
_lib.qsv_version.argtypes = []
_lib.qsv_clock.restype = C.c_double
_lib.qsv_clock.argtypes = []


def debug_inject(kind: int, count: int) -> None:
    """Failure injection for tests: kind 1 = the next `count` device
    allocations fail, kind 2 = the next `count` device calls made for a
    state fail (that state turns failed); count 0 clears."""
    _check(_lib.qsv_debug_inject(int(kind), int(count)))


def lib():
    return _lib


def last_error() -> str:
    return _lib.qsv_last_error().decode()


def version() -> str:
    return _lib.qsv_version().decode()


def _check(status: int) -> None:
    if status != QSV_OK:
        raise QsvError(status, last_error())


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


# ---------------------------------------------------------------- gates

def gate_matrix(name: str, params: Sequence[float] = ()) -> np.ndarray:
    """Standard 2x2 gate matrix from the library (complex128)."""
    p = np.asarray(params, dtype=np.float64)
    out = np.zeros(8, dtype=np.float64)
    k = C.c_int32(0)
    _check(_lib.qsv_gate_matrix(name.encode(), _ptr(p, C.c_double) if p.size
                                else None, int(p.size), _ptr(out, C.c_double),
                                C.byref(k)))
    return (out[0::2] + 1j * out[1::2]).reshape(2, 2)


def gate_matrices(name: str, params) -> np.ndarray:
    """Standard 2x2 matrices of one gate name for many parameter tuples."""
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    count = p.shape[0]
    npar = p.shape[1] if p.ndim == 2 else 0
    out = np.zeros((count, 8), dtype=np.float64)
    _check(_lib.qsv_gate_matrices(name.encode(), _ptr(p, C.c_double),
                                  npar, count, _ptr(out, C.c_double)))
    return (out[:, 0::2] + 1j * out[:, 1::2]).reshape(count, 2, 2)


class Circuit:
    """A gate list flattened into the arrays of ``qsv_circuit``."""

    def __init__(self):
        self.k, self.c, self.qubits, self.mats = [], [], [], []
        self._cache = {}

    def add(self, targets: Sequence[int], matrix, controls: Sequence[int] = ()):
        m = np.asarray(matrix, dtype=np.complex128)
        self.k.append(len(targets))
        self.c.append(len(controls))
        self.qubits.extend(int(q) for q in targets)
        self.qubits.extend(int(q) for q in controls)
        self.mats.append(np.ascontiguousarray(m).view(np.float64).reshape(-1))
        self._arrays = None
        return self

    def _std(self, name, params):
        key = (name, tuple(params))
        m = self._cache.get(key)
        if m is None:
            m = gate_matrix(name, params)
            self._cache[key] = m
        return m

    def add_named(self, name: str, qubits: Sequence[int],
                  params: Sequence[float] = ()):
        """Named gates of the synthetic workloads: one-qubit gates by name;
        cx(c, t) = X on t controlled by c; cz(a, b) = Z on b controlled by a;
        cp(a, b; l) = P(l) on b controlled by a."""
        if name == "cx":
            return self.add([qubits[1]], self._std("x", ()), [qubits[0]])
        if name == "cz":
            return self.add([qubits[1]], self._std("z", ()), [qubits[0]])
        if name == "cp":
            return self.add([qubits[1]], self._std("p", params), [qubits[0]])
        return self.add([qubits[0]], self._std(name, params))

    @classmethod
    def from_gates(cls, gates: Iterable) -> "Circuit":
        gates = list(gates)
        # parametrised gates: one library call per gate name
        mats = {}
        for name in {g.name for g in gates if g.params}:
            ps = [g.params for g in gates if g.name == name]
            base = "p" if name == "cp" else name
            mats[name] = iter(gate_matrices(base, ps))
        c = cls()
        for g in gates:
            if g.params:
                m = next(mats[g.name])
                if g.name == "cp":
                    c.add([g.qubits[1]], m, [g.qubits[0]])
                else:
                    c.add([g.qubits[0]], m)
            else:
                c.add_named(g.name, g.qubits, g.params)
        return c

    def __len__(self):
        return len(self.k)

    def arrays(self):
        if getattr(self, "_arrays", None) is None:
            k = np.asarray(self.k, dtype=np.int32)
            c = np.asarray(self.c, dtype=np.int32)
            q = np.asarray(self.qubits, dtype=np.int32)
            m = (np.concatenate(self.mats) if self.mats
                 else np.zeros(0, np.float64))
            self._arrays = (k, c, q, np.ascontiguousarray(m))
        return self._arrays

    def struct(self) -> qsv_circuit:
        k, c, q, m = self.arrays()
        return qsv_circuit(len(k), _ptr(k, C.c_int32), _ptr(c, C.c_int32),
                           _ptr(q, C.c_int32), _ptr(m, C.c_double))


def fuse_opts(strategy: int = 0, tile_log2: int = 0, k_max: int = 0,
              low_qubits: int = 0, reg_log2: int = 0) -> qsv_fuse_opts:
    return qsv_fuse_opts(strategy, tile_log2, k_max, low_qubits, reg_log2)


def plan_describe(circ: Circuit, n: int, prec: int = QSV_C64,
                  opts: Optional[qsv_fuse_opts] = None):
    """Host-only planner dry run: (gate_pass, gate_order, pass_kind,
    pass_qubits) as NumPy arrays."""
    g = max(len(circ), 1)
    gate_pass = np.zeros(g, np.int32)
    gate_order = np.zeros(g, np.int32)
    pass_kind = np.zeros(g, np.int32)
    pass_qubits = np.zeros(g, np.uint64)
    npass = C.c_int32(0)
    st = circ.struct()
    _check(_lib.qsv_plan_describe(
        C.byref(st), n, prec, C.byref(opts) if opts is not None else None,
        _ptr(gate_pass, C.c_int32), _ptr(gate_order, C.c_int32),
        _ptr(pass_kind, C.c_int32), _ptr(pass_qubits, C.c_uint64),
        C.byref(npass)))
    p = npass.value
    n_g = len(circ)
    return gate_pass[:n_g], gate_order[:n_g], pass_kind[:p], pass_qubits[:p]


def plan_program_stats(circ: Circuit, n: int, prec: int = QSV_C64,
                       opts: Optional[qsv_fuse_opts] = None) -> dict:
    """Host-only dry run of the device program: pass, tile-pass, segment,
    op and phase-block counts."""
    out = np.zeros(7, np.uint64)
    st = circ.struct()
    _check(_lib.qsv_plan_program_stats(
        C.byref(st), n, prec, C.byref(opts) if opts is not None else None,
        _ptr(out, C.c_uint64), 7))
    keys = ("passes", "tile_passes", "segments", "tile_ops", "phase_blocks",
            "block_gates", "tile_flops")
    return {k: int(v) for k, v in zip(keys, out)}


def debug_emulate_tiled(circ: Circuit, n: int, state: np.ndarray,
                        opts: Optional[qsv_fuse_opts] = None) -> np.ndarray:
    """Host emulation of the tiled device program (testing aid)."""
    v = np.ascontiguousarray(np.asarray(state, dtype=np.complex128)).copy()
    st = circ.struct()
    _check(_lib.qsv_debug_emulate_tiled(
        C.byref(st), n, C.byref(opts) if opts is not None else None,
        v.ctypes.data_as(C.POINTER(C.c_double))))
    return v


# ---------------------------------------------------------------- states

def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    h = getattr(stream, "cuda_stream", stream)
    return int(h) if h else None


class State:
    """A 2^n complex state on the device (owned, or wrapping a tensor)."""

    def __init__(self, n: int, prec: int = QSV_C64, stream=None,
                 tensor=None):
        self.n = n
        self.prec = prec
        self._h = C.c_void_p()
        self._tensor = tensor
        sh = _stream_handle(stream)
        if tensor is None:
            _check(_lib.qsv_alloc(n, prec, sh, C.byref(self._h)))
        else:
            nbytes = tensor.numel() * tensor.element_size()
            _check(_lib.qsv_wrap(n, prec, tensor.data_ptr(), nbytes, sh,
                                 C.byref(self._h)))

    @property
    def handle(self):
        return self._h

    @property
    def amp_dtype(self):
        return np.complex64 if self.prec == QSV_C64 else np.complex128

    def free(self):
        if self._h:
            _check(_lib.qsv_free(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            if self._h:
                _lib.qsv_free(self._h)
        except Exception:
            pass

    def device_ptr(self) -> int:
        p = C.c_void_p()
        _check(_lib.qsv_info(self._h, C.byref(p), None, None))
        return p.value

    def init_basis(self, index: int = 0):
        _check(_lib.qsv_init_basis(self._h, int(index)))

    def apply_gate(self, targets, matrix, controls=()):
        t = np.asarray(targets, dtype=np.int32)
        c = np.asarray(controls, dtype=np.int32)
        m = np.ascontiguousarray(np.asarray(matrix, dtype=np.complex128)
                                 ).view(np.float64).reshape(-1)
        _check(_lib.qsv_apply_gate(self._h, _ptr(t, C.c_int32), len(t),
                                   _ptr(c, C.c_int32) if len(c) else None,
                                   len(c), _ptr(m, C.c_double)))

    def apply_fused(self, circ: Circuit, opts: Optional[qsv_fuse_opts] = None):
        st = circ.struct()
        _check(_lib.qsv_apply_fused(self._h, C.byref(st),
                                    C.byref(opts) if opts is not None else None))

    def apply_fused_outputs(self, circ: Circuit,
                            opts: Optional[qsv_fuse_opts] = None,
                            probs_ptr: int = 0, probs_fp64: bool = False,
                            marg_qubits: Sequence[int] = (),
                            shots: int = 0, seed: int = 0):
        """apply_fused plus outputs folded into the last tile pass:
        returns (marginal or None, samples or None)."""
        st = circ.struct()
        mq = np.ascontiguousarray(np.asarray(marg_qubits, dtype=np.int32))
        m = len(mq)
        marg = np.zeros(1 << m, np.float64) if m else None
        smp = np.zeros(shots, np.uint64) if shots else None
        o = qsv_outputs(probs_ptr or None, 1 if probs_fp64 else 0, m,
                        _ptr(mq, C.c_int32) if m else None,
                        _ptr(marg, C.c_double) if m else None,
                        int(shots), int(seed),
                        _ptr(smp, C.c_uint64) if shots else None)
        _check(_lib.qsv_apply_fused_outputs(
            self._h, C.byref(st), C.byref(opts) if opts is not None else None,
            C.byref(o)))
        return marg, smp

    def autotune(self, circ: Circuit, opts: Optional[qsv_fuse_opts] = None,
                 max_timed: int = 0):
        """Choose the tile parameters for this circuit's structure by timing
        candidates on this state (its contents are overwritten).  Returns
        (options, best_ms, default_ms, from_cache)."""
        st = circ.struct()
        best = qsv_fuse_opts()
        bms, dms = C.c_float(0), C.c_float(0)
        cached = C.c_int32(0)
        _check(_lib.qsv_autotune_fused(
            self._h, C.byref(st), C.byref(opts) if opts is not None else None,
            int(max_timed), C.byref(best), C.byref(bms), C.byref(dms),
            C.byref(cached)))
        return best, float(bms.value), float(dms.value), bool(cached.value)

    def plan_stats(self) -> dict:
        out = np.zeros(13, np.uint64)
        _check(_lib.qsv_last_plan_stats(self._h, _ptr(out, C.c_uint64), 13))
        keys = ("passes", "gates", "alg_bytes", "tile_passes", "plain_passes",
                "fused_passes", "segments", "plan_ns", "tile_ops",
                "phase_blocks", "block_gates", "folded_outputs", "tile_flops")
        return {k: int(v) for k, v in zip(keys, out)}

    def set_profiling(self, enable: bool):
        _check(_lib.qsv_set_profiling(self._h, 1 if enable else 0))

    def pass_times(self, cap: int = 1 << 16):
        """(ms per pass, kind per pass) of the last apply_fused."""
        ms = np.zeros(cap, np.float32)
        kinds = np.zeros(cap, np.int32)
        cnt = C.c_int32(0)
        _check(_lib.qsv_pass_times(self._h, _ptr(ms, C.c_float),
                                   _ptr(kinds, C.c_int32), cap, C.byref(cnt)))
        m = min(cap, cnt.value)
        return ms[:m], kinds[:m]

    def probabilities_into(self, out_ptr: int, fp64: bool):
        _check(_lib.qsv_probabilities(self._h, out_ptr, 1 if fp64 else 0))

    def probabilities(self, fp64: bool = True):
        """Device probability vector as a torch tensor (caller-owned)."""
        import torch
        dt = torch.float64 if fp64 else torch.float32
        out = torch.empty(1 << self.n, dtype=dt, device="cuda")
        self.probabilities_into(out.data_ptr(), fp64)
        return out

    def norm(self) -> float:
        v = C.c_double(0)
        _check(_lib.qsv_norm(self._h, C.byref(v)))
        return v.value

    def renormalize(self) -> float:
        v = C.c_double(0)
        _check(_lib.qsv_renormalize(self._h, C.byref(v)))
        return v.value

    def renormalize_noalloc(self) -> float:
        """renormalize without any device allocation (fixed scratch; states
        up to 30 qubits; overlapping calls on one device race)."""
        v = C.c_double(0)
        _check(_lib.qsv_renormalize_noalloc(self._h, C.byref(v)))
        return v.value

    def marginal(self, qubits: Sequence[int]) -> np.ndarray:
        q = np.asarray(qubits, dtype=np.int32)
        out = np.zeros(1 << len(q), np.float64)
        _check(_lib.qsv_marginal(self._h, _ptr(q, C.c_int32), len(q),
                                 _ptr(out, C.c_double)))
        return out

    def sample(self, shots: int, seed: int) -> np.ndarray:
        out = np.zeros(max(int(shots), 1), np.uint64)
        _check(_lib.qsv_sample(self._h, int(shots), int(seed),
                               _ptr(out, C.c_uint64)))
        return out[:shots]

    def permute_qubits(self, perm) -> None:
        """Qubit q becomes qubit perm[q]."""
        p = np.ascontiguousarray(perm, dtype=np.int32)
        _check(_lib.qsv_permute_qubits(self._h, _ptr(p, C.c_int32)))

    def top_k(self, k: int):
        """(indices, probabilities) of the k most probable outcomes."""
        idx = np.zeros(max(int(k), 1), np.uint64)
        p = np.zeros(max(int(k), 1), np.float64)
        _check(_lib.qsv_top_k(self._h, int(k), _ptr(idx, C.c_uint64),
                              _ptr(p, C.c_double)))
        return idx[:k], p[:k]

    def expectation(self, terms) -> np.ndarray:
        """<P> for each term, a dict {qubit: 'X' | 'Y' | 'Z'}."""
        xm = np.zeros(len(terms), np.uint64)
        zm = np.zeros(len(terms), np.uint64)
        for t, term in enumerate(terms):
            for q, lab in term.items():
                if lab in ("X", "Y"):
                    xm[t] |= np.uint64(1 << q)
                if lab in ("Z", "Y"):
                    zm[t] |= np.uint64(1 << q)
        out = np.zeros(len(terms), np.float64)
        _check(_lib.qsv_expectation_pauli(self._h, len(terms),
                                          _ptr(xm, C.c_uint64),
                                          _ptr(zm, C.c_uint64),
                                          _ptr(out, C.c_double)))
        return out

    def get(self) -> np.ndarray:
        out = np.zeros(1 << self.n, self.amp_dtype)
        _check(_lib.qsv_get_amplitudes(self._h, out.ctypes.data))
        return out

    def set(self, psi: np.ndarray):
        a = np.ascontiguousarray(np.asarray(psi, dtype=self.amp_dtype))
        if a.size != 1 << self.n:
            raise ValueError("wrong length")
        _check(_lib.qsv_set_amplitudes(self._h, a.ctypes.data))

    def sync(self):
        _check(_lib.qsv_sync(self._h))


# ---------------------------------------------------------------- batches

INIT_CODE = {"0": 0, "1": 1, "+": 2, "+i": 3}
BASIS_CODE = {"I": 0, "X": 1, "Y": 2}


class Batch:
    """A planned batch of subcircuit variants for one persistent launch.

    ``variants`` are ``circuits.BatchCircuit`` records (width, gates,
    cut_inputs [(qubit, label)], cut_outputs [(qubit, basis)])."""

    def __init__(self, variants, prec: int = QSV_C64, stream=None,
                 tile_log2: int = 0, reg_log2: int = 0, grid: int = 0,
                 autotune: bool = False, use_graph: bool = False,
                 out_fp64: bool = False):
        self.count = len(variants)
        self.prec = prec
        self.out_fp64 = out_fp64
        keep = []
        arr = (qsv_variant * self.count)()
        for i, v in enumerate(variants):
            circ = Circuit.from_gates(v.gates)
            iq = np.asarray([q for q, _ in v.cut_inputs], np.int32)
            il = np.asarray([INIT_CODE[l] for _, l in v.cut_inputs], np.int32)
            oq = np.asarray([q for q, _ in v.cut_outputs], np.int32)
            ob = np.asarray([BASIS_CODE[b] for _, b in v.cut_outputs],
                            np.int32)
            keep += [circ, iq, il, oq, ob]
            arr[i].width = v.width
            arr[i].body = circ.struct()
            arr[i].n_inputs = len(iq)
            arr[i].input_qubits = _ptr(iq, C.c_int32)
            arr[i].input_labels = _ptr(il, C.c_int32)
            arr[i].n_outputs = len(oq)
            arr[i].output_qubits = _ptr(oq, C.c_int32)
            arr[i].output_bases = _ptr(ob, C.c_int32)
        opts = qsv_batch_opts(tile_log2, reg_log2, grid, int(autotune),
                              int(use_graph), int(out_fp64))
        self._h = C.c_void_p()
        _check(_lib.qsv_batch_create(arr, self.count, prec, C.byref(opts),
                                     _stream_handle(stream), C.byref(self._h)))
        del keep
        self.offsets = np.zeros(self.count + 1, np.uint64)
        _check(_lib.qsv_batch_out_offsets(self._h,
                                          _ptr(self.offsets, C.c_uint64)))

    def output(self):
        """A device buffer (torch tensor) for the ragged output."""
        import torch
        dt = torch.float64 if self.out_fp64 else torch.float32
        return torch.empty(int(self.offsets[-1]), dtype=dt, device="cuda")

    def launch(self, out) -> None:
        ptr = out.data_ptr() if hasattr(out, "data_ptr") else int(out)
        _check(_lib.qsv_batch_launch(self._h, ptr))

    def stats(self) -> dict:
        out = np.zeros(10, np.uint64)
        _check(_lib.qsv_batch_stats(self._h, _ptr(out, C.c_uint64), 10))
        keys = ("variants", "passes", "tiles", "ops", "scratch_bytes",
                "tile_log2", "reg_log2", "grid", "single_tile",
                "amp_updates")
        return {k: int(v) for k, v in zip(keys, out)}

    def free(self):
        if self._h:
            _check(_lib.qsv_batch_free(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            if self._h:
                _lib.qsv_batch_free(self._h)
        except Exception:
            pass


# ------------------------------------------------------ cut reconstruction

class CutSpec:
    """A wire-cut problem for ``qsv_cut_reconstruct``.

    ``subs`` are records with ``width`` and per-local-qubit lists
    ``out_qubit``, ``cut_in``, ``cut_out`` (e.g. ``circuits.CutSub``)."""

    def __init__(self, n_qubits: int, n_cuts: int, subs):
        self.n_qubits, self.n_cuts, self.n_sub = n_qubits, n_cuts, len(subs)
        self._w = np.asarray([sb.width for sb in subs], np.int32)
        self._oq = np.asarray([q for sb in subs for q in sb.out_qubit], np.int32)
        self._ci = np.asarray([c for sb in subs for c in sb.cut_in], np.int32)
        self._co = np.asarray([c for sb in subs for c in sb.cut_out], np.int32)
        self._s = qsv_cut_spec(self.n_sub, n_cuts, n_qubits,
                               _ptr(self._w, C.c_int32),
                               _ptr(self._oq, C.c_int32),
                               _ptr(self._ci, C.c_int32),
                               _ptr(self._co, C.c_int32))

    def workspace_bytes(self) -> int:
        out = C.c_uint64()
        _check(_lib.qsv_cut_workspace_bytes(C.byref(self._s), C.byref(out)))
        return int(out.value)


def cut_reconstruct(spec: CutSpec, probs, offsets, out, workspace=None,
                    stream=None) -> None:
    """Uncut probability vector (FP64 device tensor ``out``, 2^n entries)
    from the variant vectors in the device tensor ``probs`` (float32 or
    float64) at element ``offsets`` (subcircuit-major, canonical variant
    order)."""
    import torch
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    if workspace is None:
        workspace = torch.empty(max(1, spec.workspace_bytes()),
                                dtype=torch.uint8, device=probs.device)
    fp64 = 1 if probs.dtype == torch.float64 else 0
    _check(_lib.qsv_cut_reconstruct(
        C.byref(spec._s), probs.data_ptr(), fp64, probs.numel(),
        _ptr(off, C.c_uint64), workspace.data_ptr(), workspace.numel(),
        out.data_ptr(), _stream_handle(stream)))


# ---------------------------------------------------------------- serving

def clock() -> float:
    """The library's steady clock (seconds)."""
    return _lib.qsv_clock()


class Server:
    """Request server with admission by HBM bytes and continuous batching."""

    def __init__(self, budget_bytes: int = 0, max_batch: int = 0,
                 small_width: int = 0, n_streams: int = 0,
                 serial: bool = False):
        o = qsv_server_opts(budget_bytes, max_batch, small_width, n_streams,
                            int(serial))
        self._h = C.c_void_p()
        _check(_lib.qsv_server_create(C.byref(o), C.byref(self._h)))

    def submit(self, width: int, circ: Circuit, prec: int = QSV_C64,
               shots: int = 0, seed: int = 0) -> int:
        """Enqueue a circuit on |0..0>; shots > 0 asks for samples."""
        req = qsv_request(width, prec, circ.struct(), int(shots > 0),
                          int(shots), int(seed))
        t = C.c_uint64(0)
        _check(_lib.qsv_server_submit(self._h, C.byref(req), C.byref(t)))
        return t.value

    def wait(self, ticket: int, copy: bool = True, timeout=None):
        """(data, info) for a finished request; data is a NumPy copy of the
        probabilities (float32/float64) or samples (uint64).  With a timeout
        (seconds), raises QsvError(QSV_ERR_TIMEOUT) if it has not finished."""
        r = qsv_result()
        if timeout is None:
            st = _lib.qsv_server_wait(self._h, ticket, C.byref(r))
        else:
            st = _lib.qsv_server_wait_timeout(self._h, ticket, float(timeout),
                                              C.byref(r))
        info = {"status": r.status, "width": r.width, "prec": r.prec,
                "samples": bool(r.is_samples), "batched": bool(r.batched),
                "t_submit": r.t_submit, "t_admit": r.t_admit,
                "t_start": r.t_start, "t_done": r.t_done}
        _check(st)
        if r.is_samples:
            ct = C.c_uint64
            dt = np.uint64
        elif r.prec == QSV_C64:
            ct, dt = C.c_float, np.float32
        else:
            ct, dt = C.c_double, np.float64
        data = None
        if copy and r.n_out:
            buf = (ct * r.n_out).from_address(r.data)
            data = np.frombuffer(buf, dtype=dt).copy()
        return data, info

    def cancel(self, ticket: int):
        """Withdraw a request that has not been admitted yet."""
        _check(_lib.qsv_server_cancel(self._h, ticket))

    def release(self, ticket: int):
        _check(_lib.qsv_server_release(self._h, ticket))

    def stats(self) -> dict:
        out = np.zeros(8, np.uint64)
        _check(_lib.qsv_server_stats(self._h, _ptr(out, C.c_uint64), 8))
        keys = ("submitted", "completed", "batch_launches", "single_launches",
                "peak_reserved_bytes", "max_groups_in_flight", "rejected",
                "idle_trims")
        return {k: int(v) for k, v in zip(keys, out)}

    def close(self):
        if self._h:
            _check(_lib.qsv_server_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            if self._h:
                _lib.qsv_server_destroy(self._h)
        except Exception:
            pass
