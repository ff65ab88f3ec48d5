"""ctypes binding of libqsim (include/qsim.h): argument marshalling only.

Every step of the computation runs in the library's HIP kernels and host
planner.  The functions keep the C names without the ``qsim_`` prefix.  If
the shared library has not been built, importing this module raises, so no
caller can silently fall back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqsim.so")

OK, PENDING = 0, 1
EINVAL, ENOMEM, ETOOBIG, EAGAIN, ENOTFOUND, EDEVICE, ECANCELED, ESHUTDOWN = -1, -2, -3, -4, -5, -6, -7, -8
C64, C128 = 0, 1
MODE_AUTO, MODE_DENSE, MODE_LIGHTCONE, MODE_LIGHTCONE_FACTORED = 0, 1, 2, 3
RX, RY, RZ, CZ, CNOT, U1 = 0, 1, 2, 3, 4, 5


class QsimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class Gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint8), ("pad", ctypes.c_uint8 * 3), ("q0", ctypes.c_int32),
                ("q1", ctypes.c_int32), ("param", ctypes.c_int32), ("angle", ctypes.c_double),
                ("mat", ctypes.POINTER(ctypes.c_double))]


class Circuit(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_gates", ctypes.c_int32), ("n_params", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("gates", ctypes.POINTER(Gate))]


class Hamiltonian(ctypes.Structure):
    _fields_ = [("n_terms", ctypes.c_int32), ("pad", ctypes.c_int32), ("coeff", ctypes.POINTER(ctypes.c_double)),
                ("term_off", ctypes.POINTER(ctypes.c_int32)), ("qubits", ctypes.POINTER(ctypes.c_int32)),
                ("paulis", ctypes.POINTER(ctypes.c_uint8))]


class Options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_queue", ctypes.c_int32), ("cone_cap", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_uint64),
                ("tile_qubits", ctypes.c_int32), ("register_bits", ctypes.c_int32), ("coalesce_bits", ctypes.c_int32),
                ("dual_coalesce_bits", ctypes.c_int32), ("disable", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 3)]


OFF_FACTORED, OFF_ABSORB, OFF_ENTRY, OFF_EXIT, OFF_PRODUCT, OFF_PREFETCH, OFF_IO_REGS = 1, 2, 4, 8, 16, 32, 64
OFF_BATCH_PROBES, OFF_RELABEL, OFF_EARLY_TERMS = 128, 256, 512


class Request(ctypes.Structure):
    _fields_ = [("circuit", ctypes.POINTER(Circuit)), ("params", ctypes.POINTER(ctypes.c_double)),
                ("H", ctypes.POINTER(Hamiltonian)), ("want_grad", ctypes.c_int32), ("pad", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("submitted", "completed", "rejected", "cancelled", "failed", "steps",
                                                "launches", "inflight_bytes", "peak_inflight_bytes", "queued",
                                                "running", "pool_outstanding_bytes", "accounting_violations")]


assert ctypes.sizeof(Gate) == 32 and ctypes.sizeof(Circuit) == 24 and ctypes.sizeof(Hamiltonian) == 40
assert ctypes.sizeof(Options) == 56

EXPORTS = [
    "qsim_init", "qsim_finalize", "qsim_strerror", "qsim_last_error", "qsim_create_state", "qsim_destroy_state",
    "qsim_apply_layer", "qsim_expect", "qsim_state_to_host", "qsim_state_device_ptr", "qsim_expect_circuit",
    "qsim_expect_grad", "qsim_lightcone_sets", "qsim_plan_dense", "qsim_submit", "qsim_poll", "qsim_cancel",
    "qsim_server_stats_get", "qsim_timing_enable", "qsim_timing_get", "qsim_poll_timed", "qsim_clock",
    "qsim_copy_probe", "qsim_expect_grad_cones", "qsim_reduced_density", "qsim_plan_passes", "qsim_expect_terms",
    "qsim_coef_rows", "qsim_plan_trace",
    "qsim_expect_circuit_noalloc",
    "qsim_apply_block5",
]


def _load():
    # torch ships its own HIP runtime (same soname as the system one).  Loading
    # torch first makes this library bind to that runtime, so one process never
    # holds two HIP runtimes and torch's streams and device pointers are valid here.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libqsim.so is not built ({LIB_PATH}); run __graft_entry__.build() or "
                          "python paper_2112_10239_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, V = ctypes.POINTER, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    sig = {
        "qsim_init": (I, [P(V), P(Options)]),
        "qsim_finalize": (None, [V]),
        "qsim_strerror": (ctypes.c_char_p, [I]),
        "qsim_last_error": (ctypes.c_char_p, [V]),
        "qsim_create_state": (I, [V, I, I, I, V, V, P(V)]),
        "qsim_destroy_state": (I, [V]),
        "qsim_apply_layer": (I, [V, P(Gate), I, V, I, I]),
        "qsim_expect": (I, [V, P(Hamiltonian), P(D)]),
        "qsim_state_to_host": (I, [V, V]),
        "qsim_state_device_ptr": (I, [V, P(V)]),
        "qsim_expect_circuit": (I, [V, P(Circuit), V, I, I, P(Hamiltonian), I, I, V, P(D), P(V)]),
        "qsim_expect_terms": (I, [V, P(Circuit), V, I, I, P(Hamiltonian), I, I, V, P(D)]),
        "qsim_expect_grad": (I, [V, P(Circuit), V, I, I, P(Hamiltonian), I, V, V, P(D), P(D)]),
        "qsim_expect_grad_cones": (I, [V, P(Circuit), V, I, I, P(Hamiltonian), I, I, V, P(D), P(D)]),
        "qsim_reduced_density": (I, [V, P(ctypes.c_int32), I, V, I]),
        "qsim_lightcone_sets": (I, [P(Circuit), P(Hamiltonian), P(ctypes.c_int32), P(ctypes.c_int32), I]),
        "qsim_plan_dense": (I, [P(Circuit), P(Hamiltonian), I, P(ctypes.c_int64), P(ctypes.c_int32), I]),
        "qsim_plan_passes": (I, [V, P(Circuit), P(Hamiltonian), I, I, P(ctypes.c_int32), I, P(I)]),
        "qsim_plan_trace": (I, [V, P(Circuit), P(Hamiltonian), I, I, P(ctypes.c_int64), P(D), I, P(ctypes.c_int32), I,
                                P(I), P(I)]),
        "qsim_coef_rows": (I, [V, P(Circuit), V, I, I, I, V, ctypes.c_uint64, P(ctypes.c_uint64)]),
        "qsim_expect_circuit_noalloc": (I, [V, P(Circuit), V, I, I, P(Hamiltonian), I, V, ctypes.c_uint64, V, P(D)]),
        "qsim_apply_block5": (I, [V, P(D), I, P(D)]),
        "qsim_submit": (I, [V, P(Request), P(ctypes.c_uint64)]),
        "qsim_poll": (I, [V, ctypes.c_uint64, P(D), P(D)]),
        "qsim_cancel": (I, [V, ctypes.c_uint64]),
        "qsim_server_stats_get": (I, [V, P(ServerStats)]),
        "qsim_timing_enable": (I, [V, I]),
        "qsim_poll_timed": (I, [V, ctypes.c_uint64, P(D), P(D), P(D)]),
        "qsim_clock": (D, []),
        "qsim_copy_probe": (I, [V, ctypes.c_uint64, I, P(D)]),
        "qsim_timing_get": (I, [V, P(D), P(D), P(D), P(ctypes.c_int32), P(ctypes.c_int32), I, P(I)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def clock() -> float:
    """The library's monotonic clock (seconds), the timeline of serving timestamps."""
    return float(lib.qsim_clock())


def strerror(code: int) -> str:
    return lib.qsim_strerror(code).decode()


# ---------------------------------------------------------------------------
# marshalling of circuits and Hamiltonians
# ---------------------------------------------------------------------------

_GATE_NP = np.dtype({"names": ["kind", "q0", "q1", "param", "angle", "mat"],
                     "formats": [np.uint8, np.int32, np.int32, np.int32, np.float64, np.uint64],
                     "offsets": [Gate.kind.offset, Gate.q0.offset, Gate.q1.offset, Gate.param.offset,
                                 Gate.angle.offset, Gate.mat.offset],
                     "itemsize": ctypes.sizeof(Gate)})


class CCircuit:
    """A ctypes view of a gate list; keeps the backing arrays alive."""

    def __init__(self, n: int, gates: np.ndarray, n_params: int, mats: dict | None = None):
        self._mats = {}
        g = gates
        # filled column by column through a numpy view of the ctypes array
        rec = np.zeros(max(1, len(g)), dtype=_GATE_NP)
        if len(g):
            rec["kind"][: len(g)] = g["kind"]
            rec["q0"][: len(g)] = g["q0"]
            rec["q1"][: len(g)] = g["q1"]
            rec["param"][: len(g)] = g["param"]
            rec["angle"][: len(g)] = g["angle"]
        for i, mat in (mats or {}).items():
            if not 0 <= i < len(g):
                continue
            m = np.asarray(mat, dtype=np.complex128).reshape(2, 2)
            buf = np.empty(8, dtype=np.float64)
            buf[0::2] = m.real.ravel()
            buf[1::2] = m.imag.ravel()
            self._mats[i] = buf
            rec["mat"][i] = buf.ctypes.data
        self._rec = rec
        arr = (Gate * len(rec)).from_buffer(rec)
        self._arr = arr
        self.c = Circuit(n, len(g), n_params, 0, arr)
        self.n, self.n_params = n, n_params

    @classmethod
    def of(cls, circ) -> "CCircuit":
        """From any object with ``n``, ``gates`` (structured array), ``n_params`` and ``mats``.
        The marshalled copy is kept on the object and reused while its gate array is the
        same object with the same bytes (circuits with U1 matrices are marshalled anew)."""
        gates, mats = circ.gates, getattr(circ, "mats", None)
        hit = getattr(circ, "_qsim_marshalled", None)
        if (hit is not None and not mats and hit[0] is gates and hit[1] == (circ.n, circ.n_params)
                and hit[2] == gates.tobytes()):
            return hit[3]
        cc = cls(circ.n, gates, circ.n_params, mats)
        if not mats and isinstance(gates, np.ndarray):
            try:
                circ._qsim_marshalled = (gates, (circ.n, circ.n_params), gates.tobytes(), cc)
            except (AttributeError, TypeError):
                pass
        return cc


class CHamiltonian:
    def __init__(self, coeff, term_off, qubits, paulis):
        self._coeff = np.ascontiguousarray(coeff, dtype=np.float64)
        self._off = np.ascontiguousarray(term_off, dtype=np.int32)
        self._q = np.ascontiguousarray(qubits, dtype=np.int32)
        self._p = np.ascontiguousarray(paulis, dtype=np.uint8)
        if self._q.size == 0:
            self._q = np.zeros(1, dtype=np.int32)
            self._p = np.zeros(1, dtype=np.uint8)
        if self._coeff.size == 0:
            self._coeff = np.zeros(1)
        self.h = Hamiltonian(len(term_off) - 1, 0, self._coeff.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             self._off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             self._q.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             self._p.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))

    @classmethod
    def of(cls, H) -> "CHamiltonian":
        """The C view of H.  When H's four arrays need no conversion the view points into
        them (later in-place edits are seen) and is kept on H for as long as they are the
        same objects."""
        hit = getattr(H, "_qsim_marshalled", None)
        if (hit is not None and hit._coeff is H.coeff and hit._off is H.term_off and hit._q is H.qubits
                and hit._p is H.paulis):
            return hit
        ch = cls(H.coeff, H.term_off, H.qubits, H.paulis)
        if ch._coeff is H.coeff and ch._off is H.term_off and ch._q is H.qubits and ch._p is H.paulis:
            try:
                H._qsim_marshalled = ch
            except (AttributeError, TypeError):
                pass
        return ch


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _params(theta, rows: int, n_params: int) -> np.ndarray:
    th = np.ascontiguousarray(theta, dtype=np.float64).reshape(rows, n_params) if n_params else np.zeros((rows, 1))
    return th


def _is_device_tensor(theta) -> bool:
    return hasattr(theta, "is_cuda") and bool(theta.is_cuda)


def _torch_stream(t):
    """torch's current stream on t's device (a hipStream_t), which produced t's values."""
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _param_args(theta, n_params: int):
    """(pointer, rows, on_device, keepalive, single) for theta [P] or [B, P]: a host array,
    or a float64 contiguous device tensor (passed by pointer; its values stay on the GPU)."""
    if _is_device_tensor(theta):
        import torch

        t = theta.detach()
        if t.dtype != torch.float64:
            t = t.to(torch.float64)
        t = t.contiguous()
        single = t.dim() <= 1
        rows = 1 if single else int(t.shape[0])
        if t.numel() != rows * n_params:
            raise ValueError(f"theta has {t.numel()} values, expected {rows} x {n_params}")
        return ctypes.c_void_p(t.data_ptr() if t.numel() else 0), rows, 1, t, single
    th = np.asarray(theta, dtype=np.float64)
    single = th.ndim <= 1
    rows = 1 if single else th.shape[0]
    th = _params(th, rows, n_params)
    return th.ctypes.data_as(ctypes.c_void_p), rows, 0, th, single


# ---------------------------------------------------------------------------
# host-only calls
# ---------------------------------------------------------------------------

def lightcone_sets(circ, H):
    cc, ch = CCircuit.of(circ), CHamiltonian.of(H)
    T = ch.h.n_terms
    cap = max(1, T * circ.n)
    off = np.zeros(T + 1, dtype=np.int32)
    qs = np.zeros(cap, dtype=np.int32)
    rc = lib.qsim_lightcone_sets(ctypes.byref(cc.c), ctypes.byref(ch.h),
                                 off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                 qs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cap)
    if rc != OK:
        raise QsimError(rc, "qsim_lightcone_sets: " + strerror(rc))
    return [qs[off[t]:off[t + 1]].copy() for t in range(T)]


def plan_dense(circ, H=None, dtype: int = C64):
    """(info dict, order array [G', 4] of (pass, stage, op, gate)) for a dense plan."""
    cc = CCircuit.of(circ)
    ch = CHamiltonian.of(H) if H is not None else None
    info = np.zeros(4, dtype=np.int64)
    cap = max(1, circ.n_gates)
    order = np.zeros(cap * 4, dtype=np.int32)
    rc = lib.qsim_plan_dense(ctypes.byref(cc.c), ctypes.byref(ch.h) if ch else None, dtype,
                             info.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                             order.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cap)
    if rc != OK:
        raise QsimError(rc, "qsim_plan_dense: " + strerror(rc))
    d = dict(passes=int(info[0]), stages=int(info[1]), ops=int(info[2]), meas_passes=int(info[3]))
    return d, order.reshape(-1, 4)[: circ.n_gates].copy()


# ---------------------------------------------------------------------------
# context
# ---------------------------------------------------------------------------

class Context:
    """A libqsim context on one HIP device (device=-1: host-only, simulated serving)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, max_queue: int = 0, cone_cap: int = 0,
                 max_inflight: int = 0, tile_qubits: int = 0, register_bits: int = 0, coalesce_bits: int = 0,
                 dual_coalesce_bits: int = 0, disable: int = 0):
        self._lib = lib
        opt = Options(device=device, max_queue=max_queue, cone_cap=cone_cap, max_inflight=max_inflight,
                      hbm_budget_bytes=hbm_budget_bytes, tile_qubits=tile_qubits, register_bits=register_bits,
                      coalesce_bits=coalesce_bits, dual_coalesce_bits=dual_coalesce_bits, disable=disable)
        self._ticket_params = {}  # ticket -> n_params of its request (size of the gradient buffer)
        p = ctypes.c_void_p()
        rc = lib.qsim_init(ctypes.byref(p), ctypes.byref(opt))
        if rc != OK:
            raise QsimError(rc, "qsim_init: " + strerror(rc))
        self.ptr = p

    def close(self):
        if self.ptr:
            self._lib.qsim_finalize(self.ptr)
            self.ptr = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def last_error(self) -> str:
        return lib.qsim_last_error(self.ptr).decode()

    def _check(self, rc, what):
        if rc != OK:
            raise QsimError(rc, f"{what}: {strerror(rc)}: {self.last_error()}")

    # -- one-call evaluation ----------------------------------------------------
    def expect_circuit(self, circ, H, theta, mode: int = MODE_AUTO, dtype: int = C64, stream=None, keep=False):
        """<H> for theta [P] (float) or [B, P] ([B]); keep=True also returns a State.
        theta may be a device tensor: its values are then read on the GPU only."""
        tp, rows, dev, _hold, single = _param_args(theta, circ.n_params)
        if dev and stream is None:  # read the parameters in order after the work that wrote them
            stream = _torch_stream(_hold)
        cc, ch = CCircuit.of(circ), CHamiltonian.of(H)
        out = np.zeros(rows)
        kp = ctypes.c_void_p()
        rc = lib.qsim_expect_circuit(self.ptr, ctypes.byref(cc.c), tp, rows, dev, ctypes.byref(ch.h), mode, dtype,
                                     stream, _dptr(out), ctypes.byref(kp) if keep else None)
        self._check(rc, "qsim_expect_circuit")
        val = float(out[0]) if single else out
        if keep:
            return val, State._wrap(self, kp, circ.n, rows, dtype)
        return val

    def expect_circuit_noalloc(self, circ, H, theta, state, dtype: int = C64, stream=None):
        """Dense <H> through the allocation-free entry point: state is a caller device
        buffer (a contiguous torch tensor on the context's GPU, batch * 2^n complex of
        dtype) that holds the final states on return.  theta [P] or [B, P] as in
        expect_circuit.  Returns a float for theta [P], else an array [B]."""
        tp, rows, dev, _hold, single = _param_args(theta, circ.n_params)
        if dev and stream is None:  # read the parameters in order after the work that wrote them
            stream = _torch_stream(_hold)
        if not (_is_device_tensor(state) and state.is_contiguous()):
            raise ValueError("state must be a contiguous device tensor")
        nbytes = state.numel() * state.element_size()
        cc, ch = CCircuit.of(circ), CHamiltonian.of(H)
        out = np.zeros(rows)
        rc = lib.qsim_expect_circuit_noalloc(self.ptr, ctypes.byref(cc.c), tp, rows, dev, ctypes.byref(ch.h), dtype,
                                             ctypes.c_void_p(state.data_ptr()), nbytes, stream, _dptr(out))
        self._check(rc, "qsim_expect_circuit_noalloc")
        return float(out[0]) if single else out

    def expect_terms(self, circ, H, theta, mode: int = MODE_AUTO, dtype: int = C64, stream=None):
        """<P_t> per term (coefficients not applied): [T] for theta [P], [B, T] for [B, P]."""
        tp, rows, dev, _hold, single = _param_args(theta, circ.n_params)
        if dev and stream is None:  # read the parameters in order after the work that wrote them
            stream = _torch_stream(_hold)
        cc, ch = CCircuit.of(circ), CHamiltonian.of(H)
        T = ch.h.n_terms
        out = np.zeros((rows, max(T, 1)))
        rc = lib.qsim_expect_terms(self.ptr, ctypes.byref(cc.c), tp, rows, dev, ctypes.byref(ch.h), mode, dtype,
                                   stream, _dptr(out))
        self._check(rc, "qsim_expect_terms")
        out = out[:, :T]
        return out[0] if single else out

    def expect_grad(self, circ, H, theta, dtype: int = C64, stream=None, saved=None, want_E=True,
                    mode: int = MODE_DENSE):
        """(E [B], grad [B, P]) by the adjoint method; theta [P] or [B, P] (host, or a device
        tensor read on the GPU only).  mode: MODE_DENSE (full state), MODE_LIGHTCONE or
        MODE_LIGHTCONE_FACTORED (adjoint inside light cones)."""
        tp, rows, dev, _hold, single = _param_args(theta, circ.n_params)
        if dev and stream is None:  # read the parameters in order after the work that wrote them
            stream = _torch_stream(_hold)
        cc, ch = CCircuit.of(circ), CHamiltonian.of(H)
        E = np.zeros(rows)
        g = np.zeros((rows, max(1, circ.n_params)))
        if mode == MODE_DENSE:
            rc = lib.qsim_expect_grad(self.ptr, ctypes.byref(cc.c), tp, rows, dev, ctypes.byref(ch.h), dtype,
                                      stream, saved.ptr if saved is not None else None,
                                      _dptr(E) if want_E else None, _dptr(g))
            self._check(rc, "qsim_expect_grad")
        else:
            if saved is not None:
                raise ValueError("saved states are only used by the dense mode")
            rc = lib.qsim_expect_grad_cones(self.ptr, ctypes.byref(cc.c), tp, rows, dev, ctypes.byref(ch.h), mode,
                                            dtype, stream, _dptr(E) if want_E else None, _dptr(g))
            self._check(rc, "qsim_expect_grad_cones")
        g = g[:, : circ.n_params]
        if single:
            return float(E[0]), g[0]
        return E, g

    def plan_passes(self, circ, H, dtype: int = C64, keep: bool = False):
        """Per-pass records of the dense plan qsim_expect_circuit would launch: a list of
        dicts (flags, stages, store_stage, entry_perm, exit_perm, meas_index, grad_count, m)."""
        cc, ch = CCircuit.of(circ), CHamiltonian.of(H)
        cap = 4096
        rec = np.zeros(8 * cap, dtype=np.int32)
        cnt = ctypes.c_int()
        rc = lib.qsim_plan_passes(self.ptr, ctypes.byref(cc.c), ctypes.byref(ch.h), dtype, int(keep),
                                  rec.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cap, ctypes.byref(cnt))
        self._check(rc, "qsim_plan_passes")
        keys = ("flags", "stages", "store_stage", "entry_perm", "exit_perm", "meas_index", "grad_count", "m")
        return [dict(zip(keys, (int(v) for v in rec[8 * p:8 * p + 8]))) for p in range(cnt.value)]

    def plan_trace(self, circ, H, dtype: int = C64, keep: bool = False):
        """Stage trace of that plan: (records int64 [count, 8], coef float64 [count], srcs int32);
        see qsim_plan_trace for the record layout."""
        cc, ch = CCircuit.of(circ), CHamiltonian.of(H)
        cnt, nsrc = ctypes.c_int(), ctypes.c_int()
        rc = lib.qsim_plan_trace(self.ptr, ctypes.byref(cc.c), ctypes.byref(ch.h), dtype, int(keep), None, None, 0,
                                 None, 0, ctypes.byref(cnt), ctypes.byref(nsrc))
        if rc != ETOOBIG:
            self._check(rc, "qsim_plan_trace")
        rec = np.zeros((max(cnt.value, 1), 8), dtype=np.int64)
        coef = np.zeros(max(cnt.value, 1))
        srcs = np.zeros(max(nsrc.value, 1), dtype=np.int32)
        rc = lib.qsim_plan_trace(self.ptr, ctypes.byref(cc.c), ctypes.byref(ch.h), dtype, int(keep),
                                 rec.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 coef.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), rec.shape[0],
                                 srcs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), srcs.size, ctypes.byref(cnt),
                                 ctypes.byref(nsrc))
        self._check(rc, "qsim_plan_trace")
        return rec[:cnt.value], coef[:cnt.value], srcs[:nsrc.value]

    def coef_rows(self, circ, theta, dtype: int = C64) -> np.ndarray:
        """Raw coefficient rows of the dense gate plan (uint8 [rows, row_bytes]), built on the
        host for a host theta or by the device kernel for a device tensor."""
        tp, rows, dev, _hold, _ = _param_args(theta, circ.n_params)
        cc = CCircuit.of(circ)
        need = ctypes.c_uint64()
        rc = lib.qsim_coef_rows(self.ptr, ctypes.byref(cc.c), tp, rows, dev, dtype, None, 0, ctypes.byref(need))
        if rc != ETOOBIG:
            self._check(rc, "qsim_coef_rows")
        out = np.zeros(need.value, dtype=np.uint8)
        rc = lib.qsim_coef_rows(self.ptr, ctypes.byref(cc.c), tp, rows, dev, dtype, out.ctypes.data_as(ctypes.c_void_p),
                                need.value, ctypes.byref(need))
        self._check(rc, "qsim_coef_rows")
        return out.reshape(rows, -1)

    # -- states -------------------------------------------------------------------
    def create_state(self, n: int, batch: int = 1, dtype: int = C64, dev_buf=None, stream=None) -> "State":
        p = ctypes.c_void_p()
        rc = lib.qsim_create_state(self.ptr, n, batch, dtype, dev_buf, stream, ctypes.byref(p))
        self._check(rc, "qsim_create_state")
        return State._wrap(self, p, n, batch, dtype)

    # -- per-launch timing -----------------------------------------------------------
    def timing_enable(self, on: bool = True):
        self._check(lib.qsim_timing_enable(self.ptr, int(on)), "qsim_timing_enable")

    def timing_get(self, cap: int = 1 << 16):
        """Records of timed launches: dict of arrays ms, bytes, flags, kind."""
        ms = np.zeros(cap)
        by = np.zeros(cap)
        fp = np.zeros(cap)
        fl = np.zeros(cap, dtype=np.int32)
        kd = np.zeros(cap, dtype=np.int32)
        cnt = ctypes.c_int()
        self._check(lib.qsim_timing_get(self.ptr, _dptr(ms), _dptr(by), _dptr(fp),
                                        fl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                        kd.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cap, ctypes.byref(cnt)),
                    "qsim_timing_get")
        k = cnt.value
        return dict(ms=ms[:k], bytes=by[:k], flops=fp[:k], flags=fl[:k], kind=kd[:k])

    def copy_probe(self, nbytes: int, reps: int = 5) -> float:
        """Mean milliseconds of a plain device copy of nbytes (read nbytes + write nbytes)."""
        ms = ctypes.c_double()
        self._check(lib.qsim_copy_probe(self.ptr, nbytes, reps, ctypes.byref(ms)), "qsim_copy_probe")
        return ms.value

    # -- serving ------------------------------------------------------------------
    def submit(self, circ, H, theta, want_grad: bool = False) -> int:
        return self.submit_prepared(CCircuit.of(circ), CHamiltonian.of(H), theta, want_grad)

    def submit_prepared(self, cc: "CCircuit", ch: "CHamiltonian", theta, want_grad: bool = False) -> int:
        """Submit with marshalled inputs (the library deep-copies them)."""
        th = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1)
        if th.size == 0:
            th = np.zeros(1)
        req = Request(ctypes.pointer(cc.c), _dptr(th), ctypes.pointer(ch.h), int(want_grad), 0)
        t = ctypes.c_uint64()
        rc = lib.qsim_submit(self.ptr, ctypes.byref(req), ctypes.byref(t))
        if rc != OK:
            raise QsimError(rc, f"qsim_submit: {strerror(rc)}: {self.last_error()}")
        self._ticket_params[int(t.value)] = (cc.n_params, bool(want_grad))
        return int(t.value)

    def _grad_buffer(self, ticket: int):
        n_params, want_grad = self._ticket_params.get(ticket, (0, False))
        return np.zeros(max(1, n_params)), (n_params if want_grad else 0)

    def poll(self, ticket: int, n_params: int = 0):
        """(status, E, grad or None); the gradient buffer is sized from the submitted request."""
        E = np.zeros(1)
        g, n = self._grad_buffer(ticket)
        rc = lib.qsim_poll(self.ptr, ctypes.c_uint64(ticket), _dptr(E), _dptr(g))
        if rc != PENDING:
            self._ticket_params.pop(ticket, None)
        return rc, float(E[0]), (g[:n] if n else None)

    def poll_timed(self, ticket: int, n_params: int = 0):
        """(status, E, grad or None, (t_submit, t_admit, t_done)) on the qsim_clock() timeline."""
        E = np.zeros(1)
        g, n = self._grad_buffer(ticket)
        t = np.zeros(3)
        rc = lib.qsim_poll_timed(self.ptr, ctypes.c_uint64(ticket), _dptr(E), _dptr(g), _dptr(t))
        if rc != PENDING:
            self._ticket_params.pop(ticket, None)
        return rc, float(E[0]), (g[:n] if n else None), tuple(float(x) for x in t)

    def cancel(self, ticket: int) -> int:
        return lib.qsim_cancel(self.ptr, ctypes.c_uint64(ticket))

    def server_stats(self) -> dict:
        s = ServerStats()
        self._check(lib.qsim_server_stats_get(self.ptr, ctypes.byref(s)), "qsim_server_stats_get")
        return {k: int(getattr(s, k)) for k, _ in ServerStats._fields_}


class State:
    """A batch of device states (qsim_create_state)."""

    @classmethod
    def _wrap(cls, ctx, p, n, batch, dtype):
        s = cls.__new__(cls)
        s.ctx, s.ptr, s.n, s.batch, s.dtype = ctx, p, n, batch, dtype
        return s

    def destroy(self):
        if self.ptr:
            lib.qsim_destroy_state(self.ptr)
            self.ptr = None

    def __del__(self):  # pragma: no cover
        try:
            self.destroy()
        except Exception:
            pass

    def apply_layer(self, gates: np.ndarray, params=None, n_params: int = 0, mats=None):
        """Queue gates; params [batch, n_params] on the host, or a device tensor."""
        cc = CCircuit(self.n, gates, n_params, mats)
        tp, dev, hold = None, 0, None
        if n_params:
            if _is_device_tensor(params):
                tp, rows, dev, hold, _ = _param_args(params.reshape(self.batch, n_params), n_params)
                import torch

                torch.cuda.current_stream(hold.device).synchronize()  # the values are complete
            else:
                hold = np.ascontiguousarray(params, dtype=np.float64).reshape(self.batch, n_params)
                tp = hold.ctypes.data_as(ctypes.c_void_p)
        rc = lib.qsim_apply_layer(self.ptr, cc._arr, len(gates), tp, n_params, dev)
        del hold
        self.ctx._check(rc, "qsim_apply_layer")

    def expect(self, H) -> np.ndarray:
        ch = CHamiltonian.of(H)
        out = np.zeros(self.batch)
        self.ctx._check(lib.qsim_expect(self.ptr, ctypes.byref(ch.h), _dptr(out)), "qsim_expect")
        return out

    def apply_block5(self, u, method: int = 0) -> float:
        """Dense 32 x 32 unitary u (complex, [out j][in i], little-endian over qubits 0..4)
        on qubits 0..4: method 0 matrix cores, 1 vector ALUs.  Returns the kernel time in ms."""
        uu = np.ascontiguousarray(np.asarray(u, dtype=np.complex128).reshape(32, 32))
        ms = ctypes.c_double()
        self.ctx._check(lib.qsim_apply_block5(self.ptr, uu.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                              method, ctypes.byref(ms)), "qsim_apply_block5")
        return float(ms.value)

    def to_host(self) -> np.ndarray:
        dt = np.complex64 if self.dtype == C64 else np.complex128
        out = np.empty((self.batch, 1 << self.n), dtype=dt)
        self.ctx._check(lib.qsim_state_to_host(self.ptr, out.ctypes.data_as(ctypes.c_void_p)), "qsim_state_to_host")
        return out

    def reduced_density(self, qubits, out=None):
        """rho[b] = Tr_rest |psi_b><psi_b| over the qubits not listed; bit a of rho's
        index is qubits[a].  Returns a host array [batch, 2^m, 2^m], or fills 'out'
        (a device tensor of that many complex elements of the state's dtype)."""
        keep = np.ascontiguousarray(qubits, dtype=np.int32).reshape(-1)
        N = 1 << keep.size
        kp = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        if out is None:
            dt = np.complex64 if self.dtype == C64 else np.complex128
            host = np.empty((self.batch, N, N), dtype=dt)
            self.ctx._check(lib.qsim_reduced_density(self.ptr, kp, keep.size, host.ctypes.data_as(ctypes.c_void_p), 0),
                            "qsim_reduced_density")
            return host
        if out.numel() < self.batch * N * N or not out.is_contiguous():
            raise ValueError("out must be a contiguous device tensor of batch * 4^m complex elements")
        self.ctx._check(lib.qsim_reduced_density(self.ptr, kp, keep.size, ctypes.c_void_p(out.data_ptr()), 1),
                        "qsim_reduced_density")
        return out

    def device_ptr(self) -> int:
        p = ctypes.c_void_p()
        self.ctx._check(lib.qsim_state_device_ptr(self.ptr, ctypes.byref(p)), "qsim_state_device_ptr")
        return int(p.value or 0)
