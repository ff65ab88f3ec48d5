"""Pins of the CPU oracle against facts fixed outside it.

Every check here compares the oracle with something it does not compute
itself: closed forms of small circuits, an independent Kronecker-product
simulator, brute-force MaxCut, Clifford Pauli propagation, forward
reachability for light cones, and the exact trigonometric form of a circuit
in one rotation angle.  The paper (Sec. 1, Sec. 3) fixes what is computed:
expectation values of factorized operators after a circuit of gates, and
their gradients; the conventions behind the closed forms are the readings
listed with the design notes (little-endian qubits, exp(-i t P/2) rotations,
CNOT control on q0).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import workloads as W
from tests import pinlib


def one(h_terms):
    return W.Hamiltonian.from_terms(h_terms)


def build(n, fn):
    b = W.GateListBuilder(n)
    fn(b)
    return b.build()


# --- P1/P2: single-qubit closed forms -----------------------------------------

@pytest.mark.parametrize("t", [0.0, 0.3, 1.2, -2.0, math.pi, 2.9])
def test_p1_ry_closed_form(oracle_mod, t):
    c = build(1, lambda b: b.rot(W.RY, 0))
    assert oracle_mod.expect(c, one([(1.0, [(0, "Z")])]), [t]) == pytest.approx(math.cos(t), abs=1e-14)
    assert oracle_mod.expect(c, one([(1.0, [(0, "X")])]), [t]) == pytest.approx(math.sin(t), abs=1e-14)
    assert oracle_mod.expect(c, one([(1.0, [(0, "Y")])]), [t]) == pytest.approx(0.0, abs=1e-14)


@pytest.mark.parametrize("t,p", [(0.3, 0.7), (1.2, -2.5), (-2.0, 3.0), (2.2, 0.0)])
def test_p2_ry_then_rz(oracle_mod, t, p):
    c = build(1, lambda b: (b.rot(W.RY, 0), b.rot(W.RZ, 0)))
    th = [t, p]
    assert oracle_mod.expect(c, one([(1.0, [(0, "X")])]), th) == pytest.approx(math.sin(t) * math.cos(p), abs=1e-14)
    assert oracle_mod.expect(c, one([(1.0, [(0, "Y")])]), th) == pytest.approx(math.sin(t) * math.sin(p), abs=1e-14)
    assert oracle_mod.expect(c, one([(1.0, [(0, "Z")])]), th) == pytest.approx(math.cos(t), abs=1e-14)
    # amplitudes: RY(t)|0> = (cos t/2, sin t/2), then RZ(p) = diag(e^{-ip/2}, e^{ip/2})
    psi = oracle_mod.statevector(c, th)
    want = np.array([math.cos(t / 2) * np.exp(-0.5j * p), math.sin(t / 2) * np.exp(0.5j * p)])
    np.testing.assert_allclose(psi, want, atol=1e-15)


@pytest.mark.parametrize("t", [0.4, -1.7])
def test_rx_closed_form(oracle_mod, t):
    c = build(1, lambda b: b.rot(W.RX, 0))
    assert oracle_mod.expect(c, one([(1.0, [(0, "Y")])]), [t]) == pytest.approx(-math.sin(t), abs=1e-14)
    assert oracle_mod.expect(c, one([(1.0, [(0, "Z")])]), [t]) == pytest.approx(math.cos(t), abs=1e-14)
    assert oracle_mod.expect(c, one([(1.0, [(0, "X")])]), [t]) == pytest.approx(0.0, abs=1e-14)


# --- P3: bit order and CNOT direction ----------------------------------------

@pytest.mark.parametrize("n,q,qt", [(3, 0, 2), (4, 2, 1), (5, 4, 0)])
def test_p3_cnot_index_and_direction(oracle_mod, n, q, qt):
    c = build(n, lambda b: (b.rot(W.RY, q, fixed_angle=math.pi), b.two(W.CNOT, q, qt)))
    psi = oracle_mod.statevector(c, [])
    k = (1 << q) | (1 << qt)
    assert abs(psi[k]) == pytest.approx(1.0, abs=1e-15)
    assert np.sum(np.abs(psi) ** 2) - abs(psi[k]) ** 2 == pytest.approx(0.0, abs=1e-15)
    assert oracle_mod.expect(c, one([(1.0, [(qt, "Z")])]), []) == pytest.approx(-1.0, abs=1e-15)
    # the reverse direction does nothing when the control (qt) is 0
    c2 = build(n, lambda b: (b.rot(W.RY, q, fixed_angle=math.pi), b.two(W.CNOT, qt, q)))
    assert oracle_mod.expect(c2, one([(1.0, [(qt, "Z")])]), []) == pytest.approx(1.0, abs=1e-15)


# --- P4: Bell, GHZ and graph-state correlators --------------------------------

@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_p4_ghz(oracle_mod, n):
    def f(b):
        b.rot(W.RY, 0, fixed_angle=math.pi / 2)
        for i in range(n - 1):
            b.two(W.CNOT, i, i + 1)

    c = build(n, f)
    for i in range(n):
        assert oracle_mod.expect(c, one([(1.0, [(i, "Z")])]), []) == pytest.approx(0.0, abs=1e-14)
        assert oracle_mod.expect(c, one([(1.0, [(i, "X")])]), []) == pytest.approx(0.0, abs=1e-14)
        for j in range(i + 1, n):
            assert oracle_mod.expect(c, one([(1.0, [(i, "Z"), (j, "Z")])]), []) == pytest.approx(1.0, abs=1e-14)
    assert oracle_mod.expect(c, one([(1.0, [(i, "X") for i in range(n)])]), []) == pytest.approx(1.0, abs=1e-14)
    if n >= 2:  # <Y Y X...X> = -1 for GHZ
        ops = [(0, "Y"), (1, "Y")] + [(i, "X") for i in range(2, n)]
        assert oracle_mod.expect(c, one([(1.0, ops)]), []) == pytest.approx(-1.0, abs=1e-14)


def test_p4_cz_graph_state(oracle_mod):
    c = build(2, lambda b: (b.rot(W.RY, 0, fixed_angle=math.pi / 2), b.rot(W.RY, 1, fixed_angle=math.pi / 2),
                            b.two(W.CZ, 0, 1)))
    ex = lambda ops: oracle_mod.expect(c, one([(1.0, ops)]), [])
    assert ex([(0, "Z"), (1, "Z")]) == pytest.approx(0.0, abs=1e-14)
    assert ex([(0, "Z")]) == pytest.approx(0.0, abs=1e-14)
    assert ex([(0, "X")]) == pytest.approx(0.0, abs=1e-14)
    assert ex([(0, "X"), (1, "Z")]) == pytest.approx(1.0, abs=1e-14)
    assert ex([(0, "Z"), (1, "X")]) == pytest.approx(1.0, abs=1e-14)


# --- P5: product states at any n -----------------------------------------------

def product_tfim_closed_form(n, h, th_y, th_z):
    zz = sum(math.cos(th_y[i]) * math.cos(th_y[(i + 1) % n]) for i in range(n))
    x = h * sum(math.sin(th_y[i]) * math.cos(th_z[i]) for i in range(n))
    return zz + x


@pytest.mark.parametrize("n", [3, 12, 16])
def test_p5_product_tfim_dense(oracle_mod, n):
    def f(b):
        for q in range(n):
            b.rot(W.RY, q)
        for q in range(n):
            b.rot(W.RZ, q)

    c = build(n, f)
    th = W.angles(2 * n, [99, n])
    want = product_tfim_closed_form(n, 0.7, th[:n], th[n:])
    assert oracle_mod.expect(c, W.tfim(n, 0.7), th) == pytest.approx(want, abs=1e-12)


def test_p5_product_tfim_lightcone_n500(oracle_mod):
    n = 500

    def f(b):
        for q in range(n):
            b.rot(W.RY, q)
        for q in range(n):
            b.rot(W.RZ, q)

    c = build(n, f)
    th = W.angles(2 * n, [99, n])
    want = product_tfim_closed_form(n, 1.0, th[:n], th[n:])
    tot, _ = oracle_mod.expect_lightcone(c, W.tfim(n, 1.0), th)
    assert tot == pytest.approx(want, abs=1e-11)


# --- P6: norm and identity --------------------------------------------------------

def test_p6_norm_and_identity(oracle_mod):
    w = W.dense_tfim(n=12, depth=6)
    psi = oracle_mod.statevector(w.circuit, w.theta)
    assert np.vdot(psi, psi).real == pytest.approx(1.0, abs=1e-13)
    h = W.Hamiltonian.from_terms([(2.5, [])])
    assert oracle_mod.expect(w.circuit, h, w.theta) == pytest.approx(2.5, abs=1e-13)
    assert oracle_mod.expect(w.circuit, W.Hamiltonian.from_terms([]), w.theta) == 0.0


# --- P7: brute-force MaxCut ----------------------------------------------------------

@pytest.mark.parametrize("n", [4, 5, 6, 7, 8])
def test_p7_maxcut_bruteforce(oracle_mod, n):
    rng = np.random.default_rng([7, n])
    edges = W.random_regular3(n, rng) if n % 2 == 0 else W.gnp_half(n, rng)
    H = W.maxcut(edges)
    best = pinlib.brute_maxcut(n, edges.tolist())
    c = build(n, lambda b: [b.rot(W.RY, q) for q in range(n)])
    vals = []
    for mask in range(1 << n):
        th = np.array([math.pi if (mask >> q) & 1 else 0.0 for q in range(n)])
        e = oracle_mod.expect(c, H, th)
        s = [(-1) ** ((mask >> q) & 1) for q in range(n)]
        assert e == pytest.approx(sum(s[i] * s[j] for i, j in edges.tolist()), abs=1e-12)
        vals.append(e)
    assert min(vals) == pytest.approx(len(edges) - 2 * best, abs=1e-12)
    # random angles on an entangling circuit stay within [|E| - 2 MaxCut, |E|]
    cc = W.brickwork_ry_cz(n, 3)
    for r in range(5):
        e = oracle_mod.expect(cc, H, W.angles(cc.n_params, [7, n, r]))
        assert len(edges) - 2 * best - 1e-12 <= e <= len(edges) + 1e-12


# --- P8: independent Kronecker-product simulator ------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_p8_kronecker(oracle_mod, seed):
    rng = np.random.default_rng([8, seed])
    n = int(rng.integers(1, 7))
    c = W.random_circuit(n, 40, rng)
    th = W.angles(max(c.n_params, 1), [8, seed, 1])[: c.n_params]
    H = W.random_hamiltonian(n, 8, rng)
    psi_k = pinlib.kron_state(c, th)
    psi_o = oracle_mod.statevector(c, th)
    np.testing.assert_allclose(psi_o, psi_k, atol=1e-12)
    e_o = oracle_mod.expect(c, H, th)
    assert e_o == pytest.approx(pinlib.kron_expect(c, H, th), abs=1e-12)
    Hm = pinlib.kron_hamiltonian(H, n)
    assert np.linalg.eigvalsh(Hm).min() <= e_o + 1e-12
    _, tre, tim = oracle_mod.expect_state(n, psi_o, H)
    np.testing.assert_allclose(tim, 0.0, atol=1e-13)  # Hermitian terms give real values


def test_p8_kronecker_named_families(oracle_mod):
    for c, H in ((W.ring_ry_cz(6, 2), W.maxcut(W.random_regular3(6, np.random.default_rng(1)))),
                 (W.brickwork_ry_rz_cnot(5, 2), W.tfim(5, 0.5)),
                 (W.brickwork_ry_cz(7, 3), W.tfim(7, 1.0))):
        th = W.angles(c.n_params, [8, 100, c.n])
        assert oracle_mod.expect(c, H, th) == pytest.approx(pinlib.kron_expect(c, H, th), abs=1e-12)


# --- light-cone sets -------------------------------------------------------------------

def brickwork_cone_closed_form(n, q):
    """Depth-4 RY+CZ brickwork: the cone of Z_q is {q-3..q+4} for odd q, {q-4..q+3} for even q, clipped."""
    lo, hi = (q - 3, q + 4) if q % 2 == 1 else (q - 4, q + 3)
    return set(range(max(lo, 0), min(hi, n - 1) + 1))


def test_lightcone_sets_closed_form_c3(oracle_mod):
    w = W.lightcone_maxcut()
    sets = oracle_mod.lightcone_sets(w.circuit, w.H)
    assert len(sets) == 750
    sizes = []
    for (i, j), s in zip(w.edges.tolist(), sets):
        want = sorted(brickwork_cone_closed_form(500, i) | brickwork_cone_closed_form(500, j))
        assert s.tolist() == want
        sizes.append(len(s))
    assert max(sizes) <= 16


@pytest.mark.parametrize("seed", range(5))
def test_lightcone_sets_reachability(oracle_mod, seed):
    rng = np.random.default_rng([9, seed])
    n = int(rng.integers(4, 30))
    c = W.random_circuit(n, int(rng.integers(5, 60)), rng, kinds=(W.RY, W.RZ, W.CZ, W.CNOT))
    H = W.random_hamiltonian(n, 10, rng, max_weight=3)
    sets = oracle_mod.lightcone_sets(c, H)
    for (coeff, ops), s in zip(H.terms(), sets):
        assert s.tolist() == pinlib.reach_cone(c, [q for q, _ in ops])


# --- P9: light-cone values equal the dense state vector ----------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_p9_lightcone_equals_dense(oracle_mod, seed):
    rng = np.random.default_rng([10, seed])
    n = int(rng.integers(6, 15))
    c = W.random_circuit(n, 50, rng)
    th = W.angles(max(c.n_params, 1), [10, seed])[: c.n_params]
    H = W.random_hamiltonian(n, 12, rng)
    psi = oracle_mod.statevector(c, th)
    tot_d, tre, _ = oracle_mod.expect_state(n, psi, H)
    tot_l, tl = oracle_mod.expect_lightcone(c, H, th)
    assert tot_l == pytest.approx(tot_d, abs=1e-12)
    np.testing.assert_allclose(tl, tre, atol=1e-12)


def test_p9_brickwork_n14(oracle_mod):
    c = W.brickwork_ry_cz(14, 4)
    H = W.maxcut(W.random_regular3(14, np.random.default_rng([3, 14])))
    th = W.angles(c.n_params, [3, 14, 1])
    assert oracle_mod.expect_lightcone(c, H, th)[0] == pytest.approx(oracle_mod.expect(c, H, th), abs=1e-12)


# --- P10: Clifford instances checked by Heisenberg propagation ------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_p10_clifford_dense(oracle_mod, seed):
    rng = np.random.default_rng([11, seed])
    n = 10
    c = W.brickwork_ry_rz_cnot(n, 4) if seed % 2 == 0 else W.ring_ry_cz(n, 3)
    th = pinlib.clifford_angles(c.n_params, rng)
    H = W.tfim(n, 0.5) if seed % 2 == 0 else W.random_hamiltonian(n, 10, rng)
    want = pinlib.clifford_expect(c, H, th)
    assert oracle_mod.expect(c, H, th) == pytest.approx(want, abs=1e-12)


def test_p10_clifford_lightcone_n500(oracle_mod):
    w = W.lightcone_maxcut()
    th = pinlib.clifford_angles(w.circuit.n_params, np.random.default_rng([11, 500]))
    want = pinlib.clifford_expect(w.circuit, w.H, th)
    tot, _ = oracle_mod.expect_lightcone(w.circuit, w.H, th)
    assert tot == pytest.approx(want, abs=1e-10)
    assert abs(want - round(want)) < 1e-9  # integer-valued


# --- P11: gradients by the exact trigonometric form ---------------------------------------

def test_p11_shift_rule_and_fd(oracle_mod):
    w = W.dense_tfim(n=8, depth=3)
    th = w.theta
    idx = np.array([0, 5, 17, 30, 47], dtype=np.int32)
    psr = oracle_mod.grad_psr(w.circuit, w.H, th, idx)
    h = 1e-3
    fd = oracle_mod.grad_fd(w.circuit, w.H, th, step=h, idx=idx)
    # E(t) = A + B cos t + C sin t exactly, so central FD = dE/dt * sin(h)/h
    np.testing.assert_allclose(fd * h / math.sin(h), psr, atol=1e-9)
    # three-point fit of the trigonometric form, derivative at theta_j
    for k, j in enumerate(idx):
        vals = []
        for s in (0.0, 2 * math.pi / 3, -2 * math.pi / 3):
            t2 = th.copy()
            t2[j] += s
            vals.append(oracle_mod.expect(w.circuit, w.H, t2))
        A = np.array([[1, math.cos(th[j] + s), math.sin(th[j] + s)] for s in (0.0, 2 * math.pi / 3, -2 * math.pi / 3)])
        a, b, cc = np.linalg.solve(A, np.array(vals))
        deriv = -b * math.sin(th[j]) + cc * math.cos(th[j])
        assert psr[k] == pytest.approx(deriv, abs=1e-11)


@pytest.mark.parametrize("fam", ["ry_cz_maxcut", "ry_rz_cnot_tfim"])
def test_p11_lightcone_gradient_equals_dense(oracle_mod, fam):
    """Light-cone parameter shift = full-state parameter shift (itself pinned by the trigonometric form)."""
    if fam == "ry_cz_maxcut":
        c = W.brickwork_ry_cz(12, 4)
        H = W.maxcut(W.random_regular3(12, np.random.default_rng([3, 12])))
    else:
        c = W.brickwork_ry_rz_cnot(10, 3)
        H = W.tfim(10, 0.7)
    th = W.angles(c.n_params, [3, 12, 2])
    idx = np.arange(c.n_params, dtype=np.int32)
    np.testing.assert_allclose(oracle_mod.grad_psr_lightcone(c, H, th, idx), oracle_mod.grad_psr(c, H, th),
                               atol=1e-11)


def test_p11_lightcone_gradient_product_state_n500(oracle_mod):
    """One RY layer on 500 qubits: <Z_i Z_j> = cos t_i cos t_j, so d<H>/dt_i = -sin t_i sum_j~i cos t_j."""
    n = 500
    b = W.GateListBuilder(n)
    for q in range(n):
        b.rot(W.RY, q)
    c = b.build()
    edges = W.random_regular3(n, np.random.default_rng([3, 0]))
    H = W.maxcut(edges)
    th = W.angles(n, [3, 500, 7])
    idx = np.array([0, 17, 250, 499], dtype=np.int32)
    got = oracle_mod.grad_psr_lightcone(c, H, th, idx)
    for k, i in enumerate(idx):
        nb = [int(b_) for a_, b_ in edges if a_ == i] + [int(a_) for a_, b_ in edges if b_ == i]
        want = -math.sin(th[i]) * sum(math.cos(th[j]) for j in nb)
        assert got[k] == pytest.approx(want, abs=1e-12)


def test_p11_lightcone_gradient_clifford_n500(oracle_mod):
    """At Clifford angles both shifted points are Clifford: the shift rule from Heisenberg propagation."""
    w = W.lightcone_maxcut()
    th = pinlib.clifford_angles(w.circuit.n_params, np.random.default_rng([11, 501]))
    idx = np.array([640, 1998], dtype=np.int32)
    got = oracle_mod.grad_psr_lightcone(w.circuit, w.H, th, idx)
    for k, j in enumerate(idx):
        tp, tm = th.copy(), th.copy()
        tp[j] += math.pi / 2
        tm[j] -= math.pi / 2
        want = 0.5 * (pinlib.clifford_expect(w.circuit, w.H, tp) - pinlib.clifford_expect(w.circuit, w.H, tm))
        assert got[k] == pytest.approx(want, abs=1e-10)


def test_p11_full_gradient_vs_kronecker_product_rule(oracle_mod):
    """dE/dtheta_j by differentiating the Kronecker matrix product directly (d/dt exp(-itP/2) = -i P/2 exp(...))."""
    rng = np.random.default_rng(12)
    n = 4
    c = W.random_circuit(n, 25, rng, kinds=(W.RX, W.RY, W.RZ, W.CZ, W.CNOT), p_fixed=0.0)
    th = W.angles(c.n_params, [12, 1])
    H = W.random_hamiltonian(n, 6, rng)
    Hm = pinlib.kron_hamiltonian(H, n)
    steps = list(pinlib.circuit_unitary_steps(c, th))
    want = np.zeros(c.n_params)
    for g, row in enumerate(c.gates):
        j = int(row["param"])
        if j < 0:
            continue
        P = {W.RX: pinlib.PX, W.RY: pinlib.PY, W.RZ: pinlib.PZ}[int(row["kind"])]
        Gm = pinlib._embed({int(row["q0"]): -0.5j * P}, n)
        psi = np.zeros(1 << n, dtype=complex)
        psi[0] = 1
        dpsi = None
        for k, U in enumerate(steps):
            psi = U @ psi
            if dpsi is not None:
                dpsi = U @ dpsi
            if k == g:
                dpsi = Gm @ psi
        want[j] += 2 * np.real(psi.conj() @ Hm @ dpsi)
    np.testing.assert_allclose(oracle_mod.grad_psr(c, H, th), want, atol=1e-11)


def test_invalid_inputs_rejected(oracle_mod):
    c = build(3, lambda b: b.two(W.CZ, 0, 0))
    with pytest.raises(ValueError):
        oracle_mod.expect(c, W.tfim(3, 1.0), [])
    c = build(3, lambda b: b.rot(W.RY, 0))
    with pytest.raises(ValueError):
        oracle_mod.expect(c, one([(1.0, [(5, "Z")])]), [0.1])
    with pytest.raises(ValueError):
        oracle_mod.expect(c, one([(1.0, [(0, "Z"), (0, "X")])]), [0.1])


def test_golden_ring_maxcut_regenerates(oracle_mod):
    """The stored fixture matches what the oracle computes now (guards silent oracle changes)."""
    import json
    import os

    with open(os.path.join(os.path.dirname(__file__), "golden", "ring_maxcut_n10_d4.json")) as f:
        gold = json.load(f)
    w = W.small_ring_maxcut()
    assert w.edges.tolist() == gold["edges"]
    assert oracle_mod.expect(w.circuit, w.H, w.theta) == pytest.approx(gold["E"], abs=1e-13)
    np.testing.assert_allclose(oracle_mod.grad_psr(w.circuit, w.H, w.theta), gold["grad_psr"], atol=1e-12)


# --- reduced density matrices (partial trace) ----------------------------------------------

def _ptrace_brute(psi, n, keep):
    """Definition by enumeration: rho[i, j] = sum_k psi[x(i, k)] conj(psi[x(j, k)])."""
    m = len(keep)
    rest = [q for q in range(n) if q not in keep]
    rho = np.zeros((2 ** m, 2 ** m), dtype=complex)

    def idx(i, k):
        x = 0
        for a, q in enumerate(keep):
            x |= ((i >> a) & 1) << q
        for b, q in enumerate(rest):
            x |= ((k >> b) & 1) << q
        return x

    for i in range(2 ** m):
        for j in range(2 ** m):
            rho[i, j] = sum(psi[idx(i, k)] * np.conj(psi[idx(j, k)]) for k in range(2 ** (n - m)))
    return rho


@pytest.mark.parametrize("keep", [[0], [2, 0], [1, 3, 4], [5, 0, 2, 1], [0, 1, 2, 3, 4, 5]])
def test_partial_trace_brute_force(oracle_mod, keep):
    rng = np.random.default_rng([40, len(keep)])
    n = 6
    psi = rng.normal(size=2 ** n) + 1j * rng.normal(size=2 ** n)
    psi /= np.linalg.norm(psi)
    np.testing.assert_allclose(oracle_mod.partial_trace(psi, n, keep), _ptrace_brute(psi, n, keep), atol=1e-14)


def test_partial_trace_bell_ghz_product(oracle_mod):
    # Bell pair on qubits 0, 1: either half is I/2
    c = W.GateListBuilder(2)
    c.rot(W.RY, 0, math.pi / 2)
    c.two(W.CNOT, 0, 1)
    psi = oracle_mod.statevector(c.build(), np.zeros(0))
    for q in (0, 1):
        np.testing.assert_allclose(oracle_mod.partial_trace(psi, 2, [q]), np.eye(2) / 2, atol=1e-15)
    # GHZ_5: two kept qubits give diag(1/2, 0, 0, 1/2)
    b = W.GateListBuilder(5)
    b.rot(W.RY, 0, math.pi / 2)
    for q in range(4):
        b.two(W.CNOT, q, q + 1)
    psi = oracle_mod.statevector(b.build(), np.zeros(0))
    np.testing.assert_allclose(oracle_mod.partial_trace(psi, 5, [1, 3]), np.diag([0.5, 0, 0, 0.5]), atol=1e-15)
    # product of RY(t_q)|0>: rho = kron of [[c^2, cs], [cs, s^2]] (c = cos t/2, s = sin t/2)
    t = np.array([0.3, -1.1, 2.0, 0.7])
    b = W.GateListBuilder(4)
    for q in range(4):
        b.rot(W.RY, q)
    psi = oracle_mod.statevector(b.build(), t)
    one = [np.array([[math.cos(x / 2) ** 2, math.cos(x / 2) * math.sin(x / 2)],
                     [math.cos(x / 2) * math.sin(x / 2), math.sin(x / 2) ** 2]]) for x in t]
    # keep = [3, 1]: bit 0 of i is qubit 3, bit 1 is qubit 1 -> kron(one[1], one[3])
    np.testing.assert_allclose(oracle_mod.partial_trace(psi, 4, [3, 1]), np.kron(one[1], one[3]), atol=1e-15)


def test_partial_trace_properties(oracle_mod):
    w = W.dense_tfim(n=10, depth=3)
    psi = oracle_mod.statevector(w.circuit, w.theta)
    keep = [7, 2, 4]
    rho = oracle_mod.partial_trace(psi, 10, keep)
    assert np.trace(rho).real == pytest.approx(1.0, abs=1e-13)
    np.testing.assert_allclose(rho, rho.conj().T, atol=1e-15)
    assert np.linalg.eigvalsh(rho).min() > -1e-13
    # Pauli strings on kept qubits: Tr(rho P) = <psi|P|psi>
    rng = np.random.default_rng([41, 0])
    for _ in range(6):
        letters = rng.choice(list("IXYZ"), size=3)
        if all(x == "I" for x in letters):
            continue
        H = W.Hamiltonian.from_terms([(1.0, [(q, str(L)) for q, L in zip(keep, letters) if L != "I"])])
        mats = {"I": np.eye(2), "X": np.array([[0, 1], [1, 0]]), "Y": np.array([[0, -1j], [1j, 0]]),
                "Z": np.diag([1.0, -1.0])}
        P = np.array([[1.0]])
        for L in reversed(letters):  # bit 2 of i (keep[2]) is the most significant factor
            P = np.kron(P, mats[str(L)])
        want = oracle_mod.expect_state(10, psi, H)[0]
        assert np.trace(rho @ P).real == pytest.approx(want, abs=1e-12)
    # gates on the traced qubits leave rho unchanged
    b = W.GateListBuilder(10)
    for q in (0, 1, 3, 5, 6, 8, 9):
        b.rot(W.RX, q, 0.37 * q + 0.1)
    b.two(W.CNOT, 0, 9)
    b.two(W.CZ, 3, 5)
    psi2 = psi.copy()
    c2 = b.build()
    from tests import pinlib
    for u in pinlib.circuit_unitary_steps(c2, np.zeros(0)):
        psi2 = u @ psi2
    np.testing.assert_allclose(oracle_mod.partial_trace(psi2, 10, keep), rho, atol=1e-13)
    # keeping every qubit gives the pure state's projector
    full = oracle_mod.partial_trace(psi, 10, list(range(10)))
    np.testing.assert_allclose(full, np.outer(psi, psi.conj()), atol=1e-15)
