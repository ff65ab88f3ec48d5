"""CPU oracle for circuit expectation values and their gradients (complex128).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the library.  It shares no code with
the GPU path; only the seeded input generators in ``workloads`` serve both.

Entry points and their pins (each pinned by a CPU test against something other
than the oracle itself: closed forms, brute force, an independent Kronecker-
product simulator, Clifford Pauli propagation, the parameter-shift identity):

==========================  ================================================
``statevector``             P1-P4 closed forms, Kronecker simulator (n<=8)
``expect`` / ``expect_state``  closed forms, Kronecker, brute-force MaxCut,
                            Clifford propagation at n=30 and n=500
``lightcone_sets``          hand-derived cones of the brickwork families,
                            brute-force dependency check on random circuits
``expect_lightcone``        equal to the dense value (n<=14), Clifford n=500
``grad_psr`` / ``grad_fd``  single-parameter trigonometric identity (exact
                            shift rule; FD = derivative * sin h / h)
``grad_psr_lightcone``      equal to ``grad_psr`` (n<=12), closed-form
                            product-state gradient and Clifford shift rule
                            at n=500
``partial_trace``           Bell/GHZ closed forms, product states, kept-qubit
                            Pauli expectations equal to the full state's,
                            invariance under gates on the traced qubits,
                            brute-force sum over basis states (n<=6)
==========================  ================================================

The C source ``qsim_oracle.c`` is compiled here with gcc (``build()``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qsim_oracle.c")
_LIB = os.path.join(_HERE, "_qsim_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc + OpenMP into ``oracle/_qsim_oracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fcx-limited-range",
               "-D_DEFAULT_SOURCE", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = ctypes.CDLL(_LIB)
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _circ_args(c):
    g = c.gates
    kind = np.ascontiguousarray(g["kind"], dtype=np.uint8)
    q0 = np.ascontiguousarray(g["q0"], dtype=np.int32)
    q1 = np.ascontiguousarray(g["q1"], dtype=np.int32)
    par = np.ascontiguousarray(g["param"], dtype=np.int32)
    ang = np.ascontiguousarray(g["angle"], dtype=np.float64)
    mat = np.ascontiguousarray(c.mat_array(), dtype=np.float64)
    keep = (kind, q0, q1, par, ang, mat)
    args = [ctypes.c_int(c.n), ctypes.c_int(c.n_gates), _p(kind, ctypes.c_uint8), _p(q0, ctypes.c_int32),
            _p(q1, ctypes.c_int32), _p(par, ctypes.c_int32), _p(ang, ctypes.c_double), _p(mat, ctypes.c_double),
            ctypes.c_int(c.n_params)]
    return args, keep


def _ham_args(h):
    coeff = np.ascontiguousarray(h.coeff, dtype=np.float64)
    off = np.ascontiguousarray(h.term_off, dtype=np.int32)
    qs = np.ascontiguousarray(h.qubits, dtype=np.int32)
    ps = np.ascontiguousarray(h.paulis, dtype=np.uint8)
    if qs.size == 0:  # keep valid pointers for empty arrays
        qs = np.zeros(1, dtype=np.int32)
        ps = np.zeros(1, dtype=np.uint8)
    keep = (coeff, off, qs, ps)
    args = [ctypes.c_int(h.n_terms), _p(coeff, ctypes.c_double), _p(off, ctypes.c_int32), _p(qs, ctypes.c_int32),
            _p(ps, ctypes.c_uint8)]
    return args, keep


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(k: int) -> None:
    _load().oracle_set_num_threads(ctypes.c_int(int(k)))


def statevector(c, theta) -> np.ndarray:
    """Final state as a complex128 vector of length 2^n (qubit q = index bit q)."""
    lib = _load()
    ca, keep = _circ_args(c)
    th = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1)
    if th.size == 0:
        th = np.zeros(1)
    out = np.empty(1 << c.n, dtype=np.complex128)
    _check(lib.oracle_statevector(*ca, _p(th, ctypes.c_double), _p(out, ctypes.c_double)), "statevector")
    return out


def expect_state(n: int, psi: np.ndarray, h):
    """(total, per-term real parts, per-term imaginary parts) of <psi|H|psi>."""
    lib = _load()
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    ha, keep = _ham_args(h)
    tre = np.zeros(max(h.n_terms, 1))
    tim = np.zeros(max(h.n_terms, 1))
    tot = ctypes.c_double(0.0)
    _check(lib.oracle_expect_state(ctypes.c_int(n), _p(psi, ctypes.c_double), *ha, _p(tre, ctypes.c_double),
                                   _p(tim, ctypes.c_double), ctypes.byref(tot)), "expect_state")
    return float(tot.value), tre[: h.n_terms], tim[: h.n_terms]


def expect(c, h, theta) -> np.ndarray | float:
    """<H> for theta of shape [P] (returns float) or [B, P] (returns [B])."""
    lib = _load()
    th = np.ascontiguousarray(theta, dtype=np.float64)
    single = th.ndim <= 1
    th2 = th.reshape(1, -1) if single else th
    if th2.shape[1] == 0:
        th2 = np.zeros((th2.shape[0], 1))
    ca, k1 = _circ_args(c)
    ha, k2 = _ham_args(h)
    out = np.zeros(th2.shape[0])
    _check(lib.oracle_expect(*ca, *ha, _p(th2, ctypes.c_double), ctypes.c_int(th2.shape[0]),
                             _p(out, ctypes.c_double)), "expect")
    return float(out[0]) if single else out


def grad_psr(c, h, theta, idx=None) -> np.ndarray:
    """Parameter-shift gradient (all parameters, or the listed subset)."""
    lib = _load()
    th = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1)
    ca, k1 = _circ_args(c)
    ha, k2 = _ham_args(h)
    if idx is None:
        g = np.zeros(max(c.n_params, 1))
        _check(lib.oracle_grad_psr(*ca, *ha, _p(th, ctypes.c_double), _p(g, ctypes.c_double)), "grad_psr")
        return g[: c.n_params]
    ix = np.ascontiguousarray(idx, dtype=np.int32)
    g = np.zeros(max(ix.size, 1))
    _check(lib.oracle_grad_psr_subset(*ca, *ha, _p(th, ctypes.c_double), ctypes.c_int(ix.size),
                                      _p(ix, ctypes.c_int32), _p(g, ctypes.c_double)), "grad_psr_subset")
    return g[: ix.size]


def grad_fd(c, h, theta, step: float = 1e-3, idx=None) -> np.ndarray:
    """Central finite differences with the given step (complex128)."""
    lib = _load()
    th = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1)
    ix = np.arange(c.n_params, dtype=np.int32) if idx is None else np.ascontiguousarray(idx, dtype=np.int32)
    ca, k1 = _circ_args(c)
    ha, k2 = _ham_args(h)
    g = np.zeros(max(ix.size, 1))
    _check(lib.oracle_grad_fd(*ca, *ha, _p(th, ctypes.c_double), ctypes.c_double(step), ctypes.c_int(ix.size),
                              _p(ix, ctypes.c_int32), _p(g, ctypes.c_double)), "grad_fd")
    return g[: ix.size]


def lightcone_sets(c, h):
    """Canonical light-cone sets as a list of ascending int arrays, one per term."""
    lib = _load()
    ca, k1 = _circ_args(c)
    ha, k2 = _ham_args(h)
    cap = max(1, h.n_terms * c.n)
    off = np.zeros(h.n_terms + 1, dtype=np.int32)
    qs = np.zeros(cap, dtype=np.int32)
    _check(lib.oracle_lightcone_sets(*ca, *ha, _p(off, ctypes.c_int32), _p(qs, ctypes.c_int32), ctypes.c_int(cap)),
           "lightcone_sets")
    return [qs[off[t]:off[t + 1]].copy() for t in range(h.n_terms)]


def expect_lightcone(c, h, theta, max_cone: int = 24):
    """(total, per-term <P_t>) with every term evaluated on its own light cone."""
    lib = _load()
    th = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1)
    if th.size == 0:
        th = np.zeros(1)
    ca, k1 = _circ_args(c)
    ha, k2 = _ham_args(h)
    tv = np.zeros(max(h.n_terms, 1))
    tot = ctypes.c_double(0.0)
    _check(lib.oracle_expect_lightcone(*ca, *ha, _p(th, ctypes.c_double), ctypes.c_int(max_cone),
                                       _p(tv, ctypes.c_double), ctypes.byref(tot)), "expect_lightcone")
    return float(tot.value), tv[: h.n_terms]


def grad_psr_lightcone(c, h, theta, idx, max_cone: int = 24) -> np.ndarray:
    """Parameter-shift derivative for the listed parameters, every term on its canonical light cone."""
    lib = _load()
    th = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1)
    if th.size == 0:
        th = np.zeros(1)
    ix = np.ascontiguousarray(idx, dtype=np.int32)
    ca, k1 = _circ_args(c)
    ha, k2 = _ham_args(h)
    g = np.zeros(max(ix.size, 1))
    _check(lib.oracle_grad_psr_lightcone(*ca, *ha, _p(th, ctypes.c_double), ctypes.c_int(max_cone),
                                         ctypes.c_int(ix.size), _p(ix, ctypes.c_int32), _p(g, ctypes.c_double)),
           "grad_psr_lightcone")
    return g[: ix.size]


def partial_trace(psi, n: int, keep) -> np.ndarray:
    """Reduced density matrix of a pure state (paper, Sec. 2: partial trace as a
    contraction): rho[i, j] = sum_k psi(i, k) conj(psi(j, k)), where bit a of i
    (and j) is qubit keep[a] and k runs over the other qubits.  psi: 2^n complex
    amplitudes, qubit q = bit q of the index.  Plain numpy, complex128."""
    keep = [int(q) for q in keep]
    m = len(keep)
    rest = [q for q in range(n) if q not in keep]
    # tensor axes: axis a of reshape(2,...,2) in C order is qubit n-1-a
    t = np.asarray(psi, dtype=np.complex128).reshape((2,) * n)
    ax_keep = [n - 1 - q for q in reversed(keep)]  # most significant kept bit first
    ax_rest = [n - 1 - q for q in reversed(rest)]
    M = np.transpose(t, ax_keep + ax_rest).reshape(2 ** m, 2 ** (n - m))
    return M @ M.conj().T


if __name__ == "__main__":  # pragma: no cover
    print(build())
    sys.exit(0)
