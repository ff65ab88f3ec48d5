"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *describes* circuits, Hamiltonians and angles: gate lists,
Pauli-term lists, graphs and random numbers.  It performs none of the
simulation arithmetic (no gate matrices, no amplitudes, no expectation
values), so that the CPU oracle and the GPU path can both consume exactly the
same inputs while sharing no code that computes anything.

Conventions fixed here (the paper is silent on them; see the list of readings
kept with the design notes):

* qubit ``q`` is bit ``q`` of an amplitude index (little-endian);
* a layer applies its rotations first, then its entanglers;
* in a layer with RY and RZ, all RY gates (ascending qubit) precede all RZ
  gates (ascending qubit); one parameter per rotation gate, numbered in
  gate-list order;
* "CNOT brickwork" = even pairs (2k, 2k+1) then odd pairs (2k+1, 2k+2) in every
  layer, open chain, control on the lower qubit;
* "RY+CZ brickwork" = layer l applies CZ on the pairs (i, i+1) with
  i = l (mod 2), open chain;
* the ring ansatz applies CZ on (i, i+1 mod n) for every i;
* Hamiltonians are real-weighted Pauli strings; TFIM is periodic,
  H = sum_i Z_i Z_{i+1 mod n} + h sum_i X_i; MaxCut is H = sum_{(i,j) in E} Z_i Z_j.

Gate kinds are small integers forming the interchange format understood by
both the oracle and the library (RX=0, RY=1, RZ=2, CZ=3, CNOT=4, U1=5).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

RX, RY, RZ, CZ, CNOT, U1 = 0, 1, 2, 3, 4, 5
KIND_NAMES = {RX: "RX", RY: "RY", RZ: "RZ", CZ: "CZ", CNOT: "CNOT", U1: "U1"}
ROTATIONS = (RX, RY, RZ)
TWO_QUBIT = (CZ, CNOT)

GATE_DTYPE = np.dtype(
    [("kind", np.uint8), ("q0", np.int32), ("q1", np.int32), ("param", np.int32), ("angle", np.float64)]
)


@dataclass
class Circuit:
    """An ordered gate list on ``n`` qubits.

    ``gates`` is a structured array of ``GATE_DTYPE``.  ``param`` indexes the
    parameter vector (``-1`` = fixed ``angle``).  ``mats`` maps a gate index of
    kind U1 to its row-major complex 2x2 matrix.
    """

    n: int
    gates: np.ndarray
    n_params: int
    mats: dict = field(default_factory=dict)

    @property
    def n_gates(self) -> int:
        return int(self.gates.shape[0])

    def mat_array(self) -> np.ndarray:
        """Flat float64 array ``[n_gates, 8]`` (re, im interleaved) for U1 gates; zeros elsewhere."""
        out = np.zeros((self.n_gates, 8), dtype=np.float64)
        for g, m in self.mats.items():
            m = np.asarray(m, dtype=np.complex128).reshape(2, 2)
            out[g, 0::2] = m.real.ravel()
            out[g, 1::2] = m.imag.ravel()
        return out


@dataclass
class Hamiltonian:
    """H = sum_t coeff[t] * P_t, P_t = prod_k paulis[k] acting on qubits[k] for k in the term's slice."""

    coeff: np.ndarray  # float64 [T]
    term_off: np.ndarray  # int32 [T+1]
    qubits: np.ndarray  # int32 [term_off[-1]]
    paulis: np.ndarray  # uint8 [term_off[-1]] in {'X','Y','Z'}

    @property
    def n_terms(self) -> int:
        return int(self.coeff.shape[0])

    def terms(self):
        for t in range(self.n_terms):
            a, b = int(self.term_off[t]), int(self.term_off[t + 1])
            yield float(self.coeff[t]), [(int(self.qubits[k]), chr(int(self.paulis[k]))) for k in range(a, b)]

    def abs_coeff_sum(self) -> float:
        return float(np.abs(self.coeff).sum())

    @staticmethod
    def from_terms(terms) -> "Hamiltonian":
        """``terms``: iterable of (coeff, [(qubit, 'X'|'Y'|'Z'), ...])."""
        coeff, off, qs, ps = [], [0], [], []
        for c, ops in terms:
            coeff.append(float(c))
            for q, p in ops:
                qs.append(int(q))
                ps.append(ord(p))
            off.append(len(qs))
        return Hamiltonian(
            np.asarray(coeff, dtype=np.float64),
            np.asarray(off, dtype=np.int32),
            np.asarray(qs, dtype=np.int32),
            np.asarray(ps, dtype=np.uint8),
        )


class GateListBuilder:
    """Appends gates in order and numbers parameters by first appearance."""

    def __init__(self, n: int):
        self.n = n
        self.rows = []
        self.n_params = 0
        self.mats = {}

    def rot(self, kind: int, q: int, fixed_angle: float | None = None) -> None:
        if fixed_angle is None:
            self.rows.append((kind, q, -1, self.n_params, 0.0))
            self.n_params += 1
        else:
            self.rows.append((kind, q, -1, -1, float(fixed_angle)))

    def two(self, kind: int, a: int, b: int) -> None:
        self.rows.append((kind, a, b, -1, 0.0))

    def custom(self, q: int, mat) -> None:
        self.mats[len(self.rows)] = np.asarray(mat, dtype=np.complex128).reshape(2, 2)
        self.rows.append((U1, q, -1, -1, 0.0))

    def build(self) -> Circuit:
        return Circuit(self.n, np.array(self.rows, dtype=GATE_DTYPE), self.n_params, dict(self.mats))


# ----------------------------------------------------------------------------
# circuit families
# ----------------------------------------------------------------------------

def ring_ry_cz(n: int, depth: int) -> Circuit:
    """Hardware-efficient ring ansatz: per layer RY on every qubit, then CZ on (i, i+1 mod n)."""
    b = GateListBuilder(n)
    for _ in range(depth):
        for q in range(n):
            b.rot(RY, q)
        for i in range(n):
            b.two(CZ, i, (i + 1) % n)
    return b.build()


def brickwork_ry_rz_cnot(n: int, depth: int) -> Circuit:
    """Per layer: RY on every qubit, RZ on every qubit, CNOT on even pairs, then on odd pairs (open chain)."""
    b = GateListBuilder(n)
    for _ in range(depth):
        for q in range(n):
            b.rot(RY, q)
        for q in range(n):
            b.rot(RZ, q)
        for i in range(0, n - 1, 2):
            b.two(CNOT, i, i + 1)
        for i in range(1, n - 1, 2):
            b.two(CNOT, i, i + 1)
    return b.build()


def brickwork_ry_cz(n: int, depth: int) -> Circuit:
    """Per layer l: RY on every qubit, then CZ on pairs (i, i+1) with i = l (mod 2), open chain."""
    b = GateListBuilder(n)
    for layer in range(depth):
        for q in range(n):
            b.rot(RY, q)
        for i in range(layer % 2, n - 1, 2):
            b.two(CZ, i, i + 1)
    return b.build()


# ----------------------------------------------------------------------------
# Hamiltonians
# ----------------------------------------------------------------------------

def tfim(n: int, h: float) -> Hamiltonian:
    """Periodic 1D transverse-field Ising: sum_i Z_i Z_{i+1 mod n} + h sum_i X_i (ZZ terms first)."""
    terms = [(1.0, [(i, "Z"), ((i + 1) % n, "Z")]) for i in range(n)]
    terms += [(h, [(i, "X")]) for i in range(n)]
    return Hamiltonian.from_terms(terms)


def maxcut(edges) -> Hamiltonian:
    """MaxCut cost Hamiltonian with unit weights: sum_{(i,j) in E} Z_i Z_j."""
    return Hamiltonian.from_terms([(1.0, [(int(i), "Z"), (int(j), "Z")]) for i, j in edges])


# ----------------------------------------------------------------------------
# graphs
# ----------------------------------------------------------------------------

def random_regular3(n: int, rng: np.random.Generator, max_tries: int = 100000) -> np.ndarray:
    """Uniform simple 3-regular graph by the pairing (configuration) model with rejection.

    For odd ``n`` no 3-regular graph exists; one uniformly chosen vertex then
    gets degree 2, giving (3n-1)/2 edges.  Edges are returned canonical
    (i < j) and sorted, as an int32 array [E, 2].
    """
    if n < 4:
        raise ValueError("need n >= 4")
    deg = np.full(n, 3, dtype=np.int64)
    if n % 2 == 1:
        deg[int(rng.integers(n))] = 2
    stubs = np.repeat(np.arange(n), deg)
    for _ in range(max_tries):
        perm = rng.permutation(stubs)
        a, b = perm[0::2], perm[1::2]
        if np.any(a == b):
            continue
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        key = lo * n + hi
        if np.unique(key).size != key.size:
            continue
        e = np.stack([lo, hi], axis=1)
        e = e[np.lexsort((e[:, 1], e[:, 0]))]
        return e.astype(np.int32)
    raise RuntimeError("pairing model did not produce a simple graph")


def gnp_half(n: int, rng: np.random.Generator) -> np.ndarray:
    """G(n, 1/2): each pair (i<j) present independently with probability 1/2 (in lexicographic order)."""
    e = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < 0.5]
    return np.asarray(e, dtype=np.int32).reshape(-1, 2)


def angles(count: int, seed) -> np.ndarray:
    """``count`` angles ~ U(-pi, pi) from ``default_rng(seed)``."""
    return np.random.default_rng(seed).uniform(-math.pi, math.pi, count)


# ----------------------------------------------------------------------------
# the five named workloads
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    circuit: Circuit
    H: Hamiltonian
    theta: np.ndarray  # [P] or [B, P]
    dtype: str  # "c64" | "c128"
    edges: np.ndarray | None = None


def small_ring_maxcut() -> Workload:
    """n=10, depth 4 ring RY+CZ, MaxCut on a random 3-regular graph on 10 nodes; complex128."""
    n, depth = 10, 4
    edges = random_regular3(n, np.random.default_rng([1, 0]))
    c = ring_ry_cz(n, depth)
    return Workload("ring_maxcut_n10_d4", c, maxcut(edges), angles(c.n_params, [1, 1]), "c128", edges)


def dense_tfim(n: int = 30, depth: int = 20) -> Workload:
    """n=30, depth 20 RY+RZ+CNOT brickwork; periodic TFIM h=1.0; complex64."""
    c = brickwork_ry_rz_cnot(n, depth)
    return Workload(f"dense_tfim_n{n}_d{depth}", c, tfim(n, 1.0), angles(c.n_params, [2, 1]), "c64")


def lightcone_maxcut(n: int = 500, depth: int = 4) -> Workload:
    """n=500, depth 4 RY+CZ brickwork; MaxCut on a random 3-regular graph on n nodes; complex64."""
    edges = random_regular3(n, np.random.default_rng([3, 0]))
    c = brickwork_ry_cz(n, depth)
    return Workload(f"lightcone_maxcut_n{n}_d{depth}", c, maxcut(edges), angles(c.n_params, [3, 1]), "c64", edges)


def batched_grad_tfim(batch: int = 256, n: int = 20, depth: int = 10) -> Workload:
    """B parameter sets for n=20, depth 10 RY+RZ+CNOT brickwork; TFIM h=0.5; complex64."""
    c = brickwork_ry_rz_cnot(n, depth)
    theta = np.stack([angles(c.n_params, [4, 1, b]) for b in range(batch)])
    return Workload(f"grad_tfim_b{batch}_n{n}_d{depth}", c, tfim(n, 0.5), theta, "c64")


@dataclass
class Request:
    rid: int
    arrival_s: float
    n: int
    depth: int
    want_grad: bool
    circuit: Circuit
    H: Hamiltonian
    theta: np.ndarray


def serving_request(r: int, arrival_s: float = 0.0, n_range=(12, 28), depth_range=(4, 16)) -> Request:
    """Request ``r`` of the serving stream: random 3-regular MaxCut on RY+CZ brickwork."""
    rng = np.random.default_rng([5, 2, r])
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    depth = int(rng.integers(depth_range[0], depth_range[1] + 1))
    want_grad = bool(rng.random() < 0.5)
    edges = random_regular3(n, rng)
    c = brickwork_ry_cz(n, depth)
    theta = rng.uniform(-math.pi, math.pi, c.n_params)
    return Request(r, arrival_s, n, depth, want_grad, c, maxcut(edges), theta)


def poisson_arrivals(rate_per_s: float, duration_s: float, seed=(5, 3)) -> np.ndarray:
    """Arrival times of an open-loop Poisson stream on [0, duration_s)."""
    rng = np.random.default_rng(list(seed))
    out, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t >= duration_s:
            break
        out.append(t)
    return np.asarray(out, dtype=np.float64)


def random_circuit(n: int, n_gates: int, rng: np.random.Generator, kinds=(RX, RY, RZ, CZ, CNOT, U1),
                   p_fixed: float = 0.2) -> Circuit:
    """Random gate list over the given kinds (test input); U1 gets a random unitary 2x2."""
    b = GateListBuilder(n)
    for _ in range(n_gates):
        k = int(kinds[int(rng.integers(len(kinds)))])
        if k in ROTATIONS:
            q = int(rng.integers(n))
            if rng.random() < p_fixed:
                b.rot(k, q, fixed_angle=float(rng.uniform(-math.pi, math.pi)))
            else:
                b.rot(k, q)
        elif k in TWO_QUBIT:
            if n < 2:
                continue
            a, c = rng.choice(n, size=2, replace=False)
            b.two(k, int(a), int(c))
        else:
            z = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
            qm, r = np.linalg.qr(z)
            qm = qm * (np.diag(r) / np.abs(np.diag(r)))
            b.custom(int(rng.integers(n)), qm)
    return b.build()


def random_hamiltonian(n: int, n_terms: int, rng: np.random.Generator, max_weight: int = 3,
                       letters: str = "XYZ") -> Hamiltonian:
    """Random real-weighted Pauli strings with distinct qubits per term (test input)."""
    terms = []
    for _ in range(n_terms):
        w = int(rng.integers(1, min(max_weight, n) + 1))
        qs = rng.choice(n, size=w, replace=False)
        terms.append((float(rng.normal()), [(int(q), letters[int(rng.integers(len(letters)))]) for q in qs]))
    return Hamiltonian.from_terms(terms)
