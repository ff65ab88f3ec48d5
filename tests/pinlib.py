"""Independent checkers used to pin the oracle (test side only).

* ``kron_state`` / ``kron_expect``: every gate and every Pauli string is
  expanded to a full 2^n x 2^n matrix with numpy.kron and multiplied out
  (a different algorithm from the oracle's in-place index-pair updates).
* ``clifford_expect``: Heisenberg-picture propagation of each Pauli string
  backwards through the gates; each conjugation U^dagger P U is computed
  numerically from the gate's own matrix and decomposed in the Pauli basis,
  so no hand-written conjugation table is involved.  Exact for circuits whose
  gates map Pauli strings to signed Pauli strings (angles in (pi/2)Z).
* ``reach_cone``: light cone by forward reachability in the time-expanded
  circuit graph (the oracle uses a backward closure).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

import workloads as W

I2 = np.eye(2, dtype=complex)
PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)
PAULI = {"I": I2, "X": PX, "Y": PY, "Z": PZ}


def gate_matrix_1q(kind: int, t: float, mat=None) -> np.ndarray:
    if kind == W.U1:
        return np.asarray(mat, dtype=complex).reshape(2, 2)
    P = {W.RX: PX, W.RY: PY, W.RZ: PZ}[kind]
    # exp(-i t P/2) via the eigen-decomposition of P (independent of the closed form)
    w, v = np.linalg.eigh(P)
    return (v * np.exp(-0.5j * t * w)) @ v.conj().T


def gate_matrix_2q(kind: int) -> np.ndarray:
    """Matrix on the ordered pair (q0, q1) with basis index 2*b(q0) + b(q1)."""
    if kind == W.CZ:
        return np.diag([1, 1, 1, -1]).astype(complex)
    P0 = np.diag([1, 0]).astype(complex)
    P1 = np.diag([0, 1]).astype(complex)
    return np.kron(P0, I2) + np.kron(P1, PX)  # control = q0 (left factor)


def _embed(ops: dict, n: int) -> np.ndarray:
    """Kronecker product over qubits; qubit q is bit q, so qubit n-1 is the leftmost factor."""
    m = np.array([[1.0 + 0j]])
    for q in range(n - 1, -1, -1):
        m = np.kron(m, ops.get(q, I2))
    return m


def _embed_2q(u4: np.ndarray, a: int, b: int, n: int) -> np.ndarray:
    # expand u4 = sum_{ij} u4[2*ra+rb, 2*ca+cb] |ra rb><ca cb| on qubits (a, b)
    E = [[np.array([[1, 0], [0, 0]], dtype=complex), np.array([[0, 1], [0, 0]], dtype=complex)],
         [np.array([[0, 0], [1, 0]], dtype=complex), np.array([[0, 0], [0, 1]], dtype=complex)]]
    out = np.zeros((1 << n, 1 << n), dtype=complex)
    for ra, rb, ca, cb in itertools.product((0, 1), repeat=4):
        coef = u4[2 * ra + rb, 2 * ca + cb]
        if coef != 0:
            out += coef * _embed({a: E[ra][ca], b: E[rb][cb]}, n)
    return out


def circuit_unitary_steps(c: W.Circuit, theta):
    mats = c.mats
    for g, row in enumerate(c.gates):
        k = int(row["kind"])
        if k in W.TWO_QUBIT:
            yield _embed_2q(gate_matrix_2q(k), int(row["q0"]), int(row["q1"]), c.n)
        else:
            t = float(theta[int(row["param"])]) if int(row["param"]) >= 0 else float(row["angle"])
            yield _embed({int(row["q0"]): gate_matrix_1q(k, t, mats.get(g))}, c.n)


def kron_state(c: W.Circuit, theta) -> np.ndarray:
    psi = np.zeros(1 << c.n, dtype=complex)
    psi[0] = 1
    for U in circuit_unitary_steps(c, theta):
        psi = U @ psi
    return psi


def kron_hamiltonian(h: W.Hamiltonian, n: int) -> np.ndarray:
    Hm = np.zeros((1 << n, 1 << n), dtype=complex)
    for coeff, ops in h.terms():
        Hm += coeff * _embed({q: PAULI[p] for q, p in ops}, n)
    return Hm


def kron_expect(c: W.Circuit, h: W.Hamiltonian, theta) -> float:
    psi = kron_state(c, theta)
    return float(np.real(psi.conj() @ kron_hamiltonian(h, c.n) @ psi))


# ---------------------------------------------------------------------------
# Clifford propagation
# ---------------------------------------------------------------------------

_LETTERS = "IXYZ"


def _decompose(M: np.ndarray, k: int):
    """Decompose a 2^k x 2^k matrix into k-qubit Pauli strings; returns {letters: coeff}."""
    out = {}
    for letters in itertools.product(_LETTERS, repeat=k):
        P = np.array([[1.0 + 0j]])
        for L in letters:  # letters[0] is the high factor
            P = np.kron(P, PAULI[L])
        coef = np.trace(P.conj().T @ M) / (1 << k)
        if abs(coef) > 1e-9:
            out["".join(letters)] = coef
    return out


def _conjugate_local(U: np.ndarray, letters: str) -> tuple[complex, str]:
    """U^dagger (P) U for a local Pauli string; must be a single signed Pauli string."""
    P = np.array([[1.0 + 0j]])
    for L in letters:
        P = np.kron(P, PAULI[L])
    d = _decompose(U.conj().T @ P @ U, len(letters))
    if len(d) != 1:
        raise ValueError("gate is not Clifford for this angle")
    (key, coef), = d.items()
    return coef, key


def clifford_expect(c: W.Circuit, h: W.Hamiltonian, theta) -> float:
    total = 0.0
    gates = list(enumerate(c.gates))
    for coeff, ops in h.terms():
        pauli = {q: p for q, p in ops}
        sign = 1.0 + 0j
        for g, row in reversed(gates):
            k = int(row["kind"])
            if k in W.TWO_QUBIT:
                a, b = int(row["q0"]), int(row["q1"])
                la, lb = pauli.get(a, "I"), pauli.get(b, "I")
                if la == "I" and lb == "I":
                    continue
                coef, key = _conjugate_local(gate_matrix_2q(k), la + lb)  # 2*b(a)+b(b): a is the high factor
                sign *= coef
                for q, L in ((a, key[0]), (b, key[1])):
                    if L == "I":
                        pauli.pop(q, None)
                    else:
                        pauli[q] = L
            else:
                q = int(row["q0"])
                L = pauli.get(q, "I")
                if L == "I":
                    continue
                t = float(theta[int(row["param"])]) if int(row["param"]) >= 0 else float(row["angle"])
                coef, key = _conjugate_local(gate_matrix_1q(k, t, c.mats.get(g)), L)
                sign *= coef
                if key == "I":
                    pauli.pop(q, None)
                else:
                    pauli[q] = key
        # <0...0| P |0...0> = product of <0|sigma|0>: 1 for I and Z, 0 for X and Y
        val = 0.0 if any(L in "XY" for L in pauli.values()) else float(np.real(sign))
        total += coeff * val
    return total


def clifford_angles(count: int, rng) -> np.ndarray:
    return rng.integers(-4, 4, count) * (math.pi / 2)


# ---------------------------------------------------------------------------
# light cones by forward reachability
# ---------------------------------------------------------------------------

def reach_cone(c: W.Circuit, support) -> list[int]:
    """Qubits q such that a path from (q, time 0) reaches the support at the end of the circuit."""
    support = set(int(s) for s in support)
    out = []
    for q0 in range(c.n):
        live = {q0}  # wires influenced by qubit q0's initial state
        for row in c.gates:
            if int(row["kind"]) in W.TWO_QUBIT:
                a, b = int(row["q0"]), int(row["q1"])
                if a in live or b in live:
                    live |= {a, b}
        if live & support:
            out.append(q0)
    return out


def brute_maxcut(n: int, edges) -> int:
    best = 0
    for mask in range(1 << n):
        cut = sum(1 for i, j in edges if ((mask >> i) & 1) != ((mask >> j) & 1))
        best = max(best, cut)
    return best
