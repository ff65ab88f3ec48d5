"""GPU parity: libqsim (HIP, gfx950) against the CPU oracle on the same seeded inputs.

Tolerances: complex64 results within 1e-5 * sum|coeff| of the complex128
oracle, complex128 results within 1e-10 * sum|coeff|; light-cone qubit sets
bit-exact.  Every call goes through the C-ABI (ctypes binding).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-5
TOL128 = 1e-10


@pytest.fixture(scope="module")
def Q():
    import paper_2112_10239_amd as Q

    return Q


@pytest.fixture(scope="module")
def eng(Q):
    ctx = Q.Context(0)
    yield ctx
    ctx.close()


def tol(H, dtype):
    return (TOL64 if dtype == 0 else TOL128) * max(1.0, H.abs_coeff_sum())


def say(*a):
    print(*a, flush=True)


# --- closed forms through the library -------------------------------------------

@pytest.mark.parametrize("dtype", [0, 1])
def test_single_qubit_closed_forms(Q, eng, dtype):
    say("closed forms dtype", dtype)
    b = W.GateListBuilder(1)
    b.rot(W.RY, 0)
    b.rot(W.RZ, 0)
    c = b.build()
    for t, p in [(0.3, 0.7), (1.2, -2.5), (-2.0, 3.0)]:
        for L, want in (("X", math.sin(t) * math.cos(p)), ("Y", math.sin(t) * math.sin(p)), ("Z", math.cos(t))):
            H = W.Hamiltonian.from_terms([(1.0, [(0, L)])])
            got = eng.expect_circuit(c, H, [t, p], mode=Q.MODE_DENSE, dtype=dtype)
            assert abs(got - want) <= (2e-6 if dtype == 0 else 1e-12), (L, got, want)


@pytest.mark.parametrize("n", [2, 3, 5, 8, 15, 17])
def test_ghz(Q, eng, n):
    say("ghz", n)
    b = W.GateListBuilder(n)
    b.rot(W.RY, 0, fixed_angle=math.pi / 2)
    for i in range(n - 1):
        b.two(W.CNOT, i, i + 1)
    c = b.build()
    terms = [(1.0, [(0, "Z"), (n - 1, "Z")]), (1.0, [(i, "X") for i in range(n)]) if n <= 4 else (0.0, [(0, "Z")]),
             (1.0, [(n // 2, "Z")]), (1.0, [(n - 1, "X")])]
    H = W.Hamiltonian.from_terms(terms)
    vals = [eng.expect_circuit(c, W.Hamiltonian.from_terms([t]), [], mode=Q.MODE_DENSE) for t in terms]
    assert vals[0] == pytest.approx(1.0, abs=1e-6)
    if n <= 4:
        assert vals[1] == pytest.approx(1.0, abs=1e-6)
    assert vals[2] == pytest.approx(0.0, abs=1e-6)
    assert vals[3] == pytest.approx(0.0, abs=1e-6)
    assert eng.expect_circuit(c, H, [], mode=Q.MODE_DENSE) == pytest.approx(sum(t[0] * v for t, v in zip(terms, vals)),
                                                                           abs=1e-6)


# --- the small named workload in complex128 -----------------------------------------

def test_ring_maxcut_n10_c128(Q, eng, oracle_mod):
    w = W.small_ring_maxcut()
    say("ring maxcut n10 c128")
    want = oracle_mod.expect(w.circuit, w.H, w.theta)
    got = eng.expect_circuit(w.circuit, w.H, w.theta, mode=Q.MODE_DENSE, dtype=Q.C128)
    assert abs(got - want) <= tol(w.H, 1), (got, want)
    got64 = eng.expect_circuit(w.circuit, w.H, w.theta, mode=Q.MODE_DENSE, dtype=Q.C64)
    assert abs(got64 - want) <= tol(w.H, 0)


# --- dense brickwork family ---------------------------------------------------------

@pytest.mark.parametrize("n,depth", [(6, 3), (10, 20), (14, 10), (15, 8), (16, 12), (19, 6), (20, 6), (20, 20), (21, 5)])
def test_dense_tfim_family(Q, eng, oracle_mod, n, depth):
    say("dense tfim", n, depth)
    c = W.brickwork_ry_rz_cnot(n, depth)
    H = W.tfim(n, 1.0)
    th = W.angles(c.n_params, [2, 1, n, depth])
    want = oracle_mod.expect(c, H, th)
    got = eng.expect_circuit(c, H, th, mode=Q.MODE_DENSE)
    assert abs(got - want) <= tol(H, 0), (got, want)


@pytest.mark.parametrize("seed", range(8))
def test_random_circuits_all_kinds(Q, eng, oracle_mod, seed):
    rng = np.random.default_rng([20, seed])
    n = int(rng.integers(1, 19))
    c = W.random_circuit(n, int(rng.integers(1, 120)), rng)
    th = W.angles(max(c.n_params, 1), [20, seed, 1])[: c.n_params]
    H = W.random_hamiltonian(n, 12, rng, max_weight=min(n, 4))
    say("random", seed, "n", n, "gates", c.n_gates)
    want = oracle_mod.expect(c, H, th)
    for dtype in (0, 1):
        got = eng.expect_circuit(c, H, th, mode=Q.MODE_DENSE, dtype=dtype)
        assert abs(got - want) <= tol(H, dtype), (dtype, got, want)


@pytest.mark.parametrize("n", [1, 4, 9, 16, 18])
def test_amplitudes(Q, eng, oracle_mod, n):
    say("amplitudes", n)
    rng = np.random.default_rng([21, n])
    c = W.random_circuit(n, 60, rng)
    th = W.angles(max(c.n_params, 1), [21, n])[: c.n_params]
    psi_o = oracle_mod.statevector(c, th)
    st = eng.create_state(n, batch=1, dtype=Q.C128)
    st.apply_layer(c.gates, th, c.n_params, mats=c.mats)
    psi = st.to_host()[0]
    st.destroy()
    np.testing.assert_allclose(psi, psi_o, atol=1e-12)


def _rotation_mix(n, depth, seed):
    """Brickwork of RY RZ (+ RX on some layers, a fixed U1 on others) and CNOTs with
    angles that include exact multiples of pi/2: every form of the factored rotation
    (tan form, swapped form, k = 0, pre-diagonal) appears."""
    rng = np.random.default_rng([24, seed])
    b = W.GateListBuilder(n)
    special = [0.0, math.pi, -math.pi, math.pi / 2, 3 * math.pi, 2.0, -2.0]
    h = np.array([[1, 1], [1, -1]]) / math.sqrt(2)
    for layer in range(depth):
        for q in range(n):
            if layer % 3 == 2 and q % 2 == 0:
                b.rot(W.RX, q, fixed_angle=float(special[(q + layer) % len(special)]))
            else:
                b.rot(W.RY, q, fixed_angle=float(special[(q + layer) % len(special)]) if q % 3 == 0 else None)
            b.rot(W.RZ, q)
            if layer == 1 and q % 4 == 1:
                b.custom(q, h if q % 8 == 1 else np.array([[0, 1], [1, 0]]))
        for q in range(layer % 2, n - 1, 2):
            b.two(W.CNOT, q, q + 1)
    c = b.build()
    th = rng.uniform(-math.pi, math.pi, c.n_params)
    th[::5] = math.pi
    return c, th


@pytest.mark.parametrize("n", [2, 5, 13, 14, 17])
def test_rotation_forms_amplitudes_c64(Q, eng, oracle_mod, n):
    """complex64 amplitudes element by element against the oracle's state vector,
    across tiles and passes (stores and exchanges of swapped registers)."""
    c, th = _rotation_mix(n, 6, n)
    say("rotation forms amplitudes", n, "gates", c.n_gates)
    psi_o = oracle_mod.statevector(c, th)
    st = eng.create_state(n, batch=1, dtype=Q.C64)
    st.apply_layer(c.gates, th, c.n_params, mats=c.mats)
    psi = st.to_host()[0]
    st.destroy()
    np.testing.assert_allclose(psi, psi_o, atol=2e-6)


@pytest.mark.parametrize("n", [1, 3, 14])
def test_rotation_forms_measured_c64(Q, eng, oracle_mod, n):
    """measurement terms on the register bits of a stage ending in rotations"""
    c, th = _rotation_mix(n, 3, 100 + n)
    terms = [(0.7, [(q, "Z")]) for q in range(n)] + [(0.3, [(q, "X")]) for q in range(n)]
    terms += [(0.2, [(q, "Y"), ((q + 1) % n, "Z")]) for q in range(n - 1)]
    H = W.Hamiltonian.from_terms(terms)
    say("rotation forms measured", n)
    want = oracle_mod.expect(c, H, th)
    got = eng.expect_circuit(c, H, th, mode=Q.MODE_DENSE, dtype=0)
    assert abs(got - want) <= tol(H, 0), (got, want)


def test_nonunitary_u1_rejected(Q, eng):
    b = W.GateListBuilder(2)
    b.custom(0, np.array([[1.0, 0.0], [0.0, 0.5]]))
    with pytest.raises(Q.QsimError) as ei:
        eng.expect_circuit(b.build(), W.tfim(2, 1.0), [], mode=Q.MODE_DENSE)
    assert ei.value.code == -1


def test_batched_rows_and_layers(Q, eng, oracle_mod):
    n, depth, B = 12, 4, 5
    c = W.brickwork_ry_rz_cnot(n, depth)
    H = W.tfim(n, 0.5)
    th = np.stack([W.angles(c.n_params, [22, b]) for b in range(B)])
    say("batched rows")
    want = oracle_mod.expect(c, H, th)
    got = eng.expect_circuit(c, H, th, mode=Q.MODE_DENSE)
    np.testing.assert_allclose(got, want, atol=tol(H, 0))
    # same circuit applied layer by layer through the stateful interface
    st = eng.create_state(n, batch=B)
    per_layer = len(c.gates) // depth
    ppl = c.n_params // depth
    for layer in range(depth):
        g = c.gates[layer * per_layer:(layer + 1) * per_layer].copy()
        g["param"] = np.where(g["param"] >= 0, g["param"] - layer * ppl, -1)
        st.apply_layer(g, th[:, layer * ppl:(layer + 1) * ppl], ppl)
    np.testing.assert_allclose(st.expect(H), want, atol=tol(H, 0))
    st.destroy()


def test_edge_cases(Q, eng, oracle_mod):
    say("edge cases")
    c = W.brickwork_ry_cz(7, 2)
    th = W.angles(c.n_params, [23])
    # empty Hamiltonian, identity only
    assert eng.expect_circuit(c, W.Hamiltonian.from_terms([]), th, mode=Q.MODE_DENSE) == 0.0
    assert eng.expect_circuit(c, W.Hamiltonian.from_terms([(2.5, [])]), th, mode=Q.MODE_DENSE) == 2.5
    # no gates
    e = W.GateListBuilder(5).build()
    assert eng.expect_circuit(e, W.tfim(5, 1.0), [], mode=Q.MODE_DENSE) == pytest.approx(5.0, abs=1e-6)
    # invalid inputs are rejected with EINVAL
    bad = W.GateListBuilder(3)
    bad.two(W.CZ, 1, 1)
    with pytest.raises(Q.QsimError) as ei:
        eng.expect_circuit(bad.build(), W.tfim(3, 1.0), [], mode=Q.MODE_DENSE)
    assert ei.value.code == -1


# --- light cones ---------------------------------------------------------------------

@pytest.mark.parametrize("n", [8, 12, 14])
def test_lightcone_equals_dense(Q, eng, oracle_mod, n):
    say("lightcone vs dense", n)
    c = W.brickwork_ry_cz(n, 4)
    H = W.maxcut(W.random_regular3(n, np.random.default_rng([24, n])))
    th = W.angles(c.n_params, [24, n, 1])
    want = oracle_mod.expect(c, H, th)
    lc = eng.expect_circuit(c, H, th, mode=Q.MODE_LIGHTCONE)
    de = eng.expect_circuit(c, H, th, mode=Q.MODE_DENSE)
    assert abs(lc - want) <= tol(H, 0)
    assert abs(de - want) <= tol(H, 0)


def test_lightcone_random_terms(Q, eng, oracle_mod):
    rng = np.random.default_rng(25)
    n = 13
    c = W.random_circuit(n, 70, rng)
    th = W.angles(max(c.n_params, 1), [25])[: c.n_params]
    H = W.random_hamiltonian(n, 10, rng, max_weight=3)
    say("lightcone random terms")
    want = oracle_mod.expect(c, H, th)
    assert abs(eng.expect_circuit(c, H, th, mode=Q.MODE_LIGHTCONE) - want) <= tol(H, 0)


def test_lightcone_n500_vs_oracle(Q, eng, oracle_mod):
    w = W.lightcone_maxcut()
    say("lightcone n500")
    sets = Q.lightcone_sets(w.circuit, w.H)
    ref = oracle_mod.lightcone_sets(w.circuit, w.H)
    assert all(np.array_equal(a, b) for a, b in zip(sets, ref))
    want, _ = oracle_mod.expect_lightcone(w.circuit, w.H, w.theta)
    got = eng.expect_circuit(w.circuit, w.H, w.theta, mode=Q.MODE_LIGHTCONE)
    assert abs(got - want) <= tol(w.H, 0), (got, want)


def test_lightcone_clifford_n500(Q, eng):
    from tests import pinlib

    w = W.lightcone_maxcut()
    th = pinlib.clifford_angles(w.circuit.n_params, np.random.default_rng([11, 500]))
    say("lightcone clifford n500")
    want = pinlib.clifford_expect(w.circuit, w.H, th)
    got = eng.expect_circuit(w.circuit, w.H, th, mode=Q.MODE_LIGHTCONE)
    assert abs(got - want) <= 1e-3, (got, want)


def test_product_state_n30_dense(Q, eng):
    """No entanglers at n=30: closed form sum cos cos + h sum sin cos (dense 8 GiB state)."""
    n = 30
    b = W.GateListBuilder(n)
    for q in range(n):
        b.rot(W.RY, q)
    for q in range(n):
        b.rot(W.RZ, q)
    c = b.build()
    th = W.angles(2 * n, [99, n])
    want = sum(math.cos(th[i]) * math.cos(th[(i + 1) % n]) for i in range(n)) + sum(
        math.sin(th[i]) * math.cos(th[n + i]) for i in range(n))
    say("product state n30")
    got = eng.expect_circuit(c, W.tfim(n, 1.0), th, mode=Q.MODE_DENSE)
    assert abs(got - want) <= 1e-5 * 60


def test_clifford_n30_dense(Q, eng):
    """Dense n=30 brickwork with Clifford angles against Heisenberg propagation (exact integers)."""
    from tests import pinlib

    w = W.dense_tfim()
    th = pinlib.clifford_angles(w.circuit.n_params, np.random.default_rng([26, 30]))
    want = pinlib.clifford_expect(w.circuit, w.H, th)
    say("clifford n30 dense")
    got = eng.expect_circuit(w.circuit, w.H, th, mode=Q.MODE_DENSE)
    assert abs(got - want) <= 1e-5 * 60, (got, want)


# --- gradients -------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_grad_random_vs_psr(Q, eng, oracle_mod, seed):
    rng = np.random.default_rng([27, seed])
    n = int(rng.integers(2, 15))
    c = W.random_circuit(n, 50, rng, p_fixed=0.1)
    th = W.angles(max(c.n_params, 1), [27, seed])[: c.n_params]
    H = W.random_hamiltonian(n, 8, rng, max_weight=min(n, 3))
    say("grad random", seed, n, c.n_params)
    psr = oracle_mod.grad_psr(c, H, th)
    E, g = eng.expect_grad(c, H, th)
    assert abs(E - oracle_mod.expect(c, H, th)) <= tol(H, 0)
    np.testing.assert_allclose(g, psr, atol=tol(H, 0))


def test_grad_tfim_batch_subset(Q, eng, oracle_mod):
    """The batched n=20 workload: rows 0-1 on a subset of parameters, shift rule and FD (h=1e-3)."""
    w = W.batched_grad_tfim(batch=8)
    c, H = w.circuit, w.H
    say("grad tfim n20 batch 8")
    E, g = eng.expect_grad(c, H, w.theta)
    idx = np.array([0, 7, 19, 20, 39, 200, 321, 399], dtype=np.int32)
    for row in (0, 1):
        psr = oracle_mod.grad_psr(c, H, w.theta[row], idx)
        np.testing.assert_allclose(g[row, idx], psr, atol=tol(H, 0))
        fd = oracle_mod.grad_fd(c, H, w.theta[row], 1e-3, idx) * (1e-3 / math.sin(1e-3))
        np.testing.assert_allclose(g[row, idx], fd, atol=tol(H, 0))
    np.testing.assert_allclose(E[:2], oracle_mod.expect(c, H, w.theta[:2]), atol=tol(H, 0))


def test_grad_saved_state_matches(Q, eng):
    w = W.batched_grad_tfim(batch=3, n=12, depth=4)
    E0, st = eng.expect_circuit(w.circuit, w.H, w.theta, mode=Q.MODE_DENSE, keep=True)
    E1, g1 = eng.expect_grad(w.circuit, w.H, w.theta, saved=st)
    st.destroy()
    E2, g2 = eng.expect_grad(w.circuit, w.H, w.theta)
    # E1 is re-measured from the kept state with a different tiling: same value up to fp32 summation order
    np.testing.assert_allclose(E1, E0, atol=tol(w.H, 0))
    # the same plans on the same inputs give the same bits
    np.testing.assert_array_equal(E2, E0)
    np.testing.assert_array_equal(g1, g2)


def test_autograd_function(Q, eng, oracle_mod):
    import torch

    from paper_2112_10239_amd.autograd import expectation

    w = W.batched_grad_tfim(batch=3, n=10, depth=3)
    theta = torch.tensor(w.theta, dtype=torch.float64, device="cuda:0", requires_grad=True)
    E = expectation(theta, eng, w.circuit, w.H)
    (E * torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64, device="cuda:0")).sum().backward()
    for row, wt in enumerate((1.0, -2.0, 0.5)):
        psr = oracle_mod.grad_psr(w.circuit, w.H, w.theta[row])
        np.testing.assert_allclose(theta.grad[row].cpu().numpy(), wt * psr, atol=tol(w.H, 0) * 2)


# --- serving ---------------------------------------------------------------------------

def test_serving_alone_equals_mix(Q, eng, oracle_mod):
    reqs = [W.serving_request(r, n_range=(12, 18), depth_range=(4, 8)) for r in range(24)]
    say("serving mix")
    alone = {}
    for r in reqs[:6]:
        t = eng.submit(r.circuit, r.H, r.theta, r.want_grad)
        while True:
            st, E, g = eng.poll(t, r.circuit.n_params)
            if st != 1:
                break
        assert st == 0
        alone[r.rid] = (E, g)
    tickets = [(r, eng.submit(r.circuit, r.H, r.theta, r.want_grad)) for r in reqs]
    res = {}
    pending = dict((t, r) for r, t in tickets)
    while pending:
        for t, r in list(pending.items()):
            st, E, g = eng.poll(t, r.circuit.n_params)
            if st == 1:
                continue
            assert st == 0, st
            res[r.rid] = (E, g)
            del pending[t]
    for rid, (E, g) in alone.items():
        assert res[rid][0] == pytest.approx(E, abs=1e-12)
        if g is not None:
            np.testing.assert_allclose(res[rid][1], g, atol=1e-12)
    for r in reqs[:8]:
        want = oracle_mod.expect(r.circuit, r.H, r.theta)
        assert abs(res[r.rid][0] - want) <= tol(r.H, 0)
        if r.want_grad:
            idx = np.arange(0, r.circuit.n_params, max(1, r.circuit.n_params // 6), dtype=np.int32)
            psr = oracle_mod.grad_psr(r.circuit, r.H, r.theta, idx)
            np.testing.assert_allclose(res[r.rid][1][idx], psr, atol=tol(r.H, 0))


def test_ring_maxcut_golden_fixture(Q, eng):
    """The library against the stored oracle fixture (complex128 energy and shift-rule gradient)."""
    import json
    import os

    with open(os.path.join(os.path.dirname(__file__), "golden", "ring_maxcut_n10_d4.json")) as f:
        gold = json.load(f)
    w = W.small_ring_maxcut()
    E = eng.expect_circuit(w.circuit, w.H, w.theta, mode=Q.MODE_DENSE, dtype=Q.C128)
    assert abs(E - gold["E"]) <= TOL128 * 15
    E2, g = eng.expect_grad(w.circuit, w.H, w.theta, dtype=Q.C128)
    assert abs(E2 - gold["E"]) <= TOL128 * 15
    np.testing.assert_allclose(g, gold["grad_psr"], atol=TOL128 * 15)


# --- factored light cones (trailing diagonal gates dropped, disjoint factors) -------------

def test_factored_n500_vs_oracle(Q, eng, oracle_mod):
    w = W.lightcone_maxcut()
    say("factored lightcone n500")
    want, _ = oracle_mod.expect_lightcone(w.circuit, w.H, w.theta)
    got = eng.expect_circuit(w.circuit, w.H, w.theta, mode=Q.MODE_LIGHTCONE_FACTORED)
    assert abs(got - want) <= tol(w.H, 0), (got, want)
    # AUTO picks the factored mode above 30 qubits
    assert eng.expect_circuit(w.circuit, w.H, w.theta) == pytest.approx(got, abs=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_factored_random_vs_dense(Q, eng, oracle_mod, seed):
    rng = np.random.default_rng([28, seed])
    n = int(rng.integers(5, 15))
    c = W.random_circuit(n, 60, rng, kinds=(W.RX, W.RY, W.RZ, W.CZ, W.CNOT))
    th = W.angles(max(c.n_params, 1), [28, seed])[: c.n_params]
    letters = "Z" if seed % 2 == 0 else "XYZ"
    H = W.random_hamiltonian(n, 10, rng, max_weight=3, letters=letters)
    say("factored random", seed, n)
    want = oracle_mod.expect(c, H, th)
    assert abs(eng.expect_circuit(c, H, th, mode=Q.MODE_LIGHTCONE_FACTORED) - want) <= tol(H, 0)


def test_factored_brickwork_clifford_n200(Q, eng):
    from tests import pinlib

    c = W.brickwork_ry_cz(200, 5)
    H = W.maxcut(W.random_regular3(200, np.random.default_rng([29, 200])))
    th = pinlib.clifford_angles(c.n_params, np.random.default_rng([29, 1]))
    say("factored clifford n200")
    want = pinlib.clifford_expect(c, H, th)
    assert abs(eng.expect_circuit(c, H, th, mode=Q.MODE_LIGHTCONE_FACTORED) - want) <= 1e-3


# --- light-cone gradients (adjoint inside every cone, weighted per-parameter sums) --------

@pytest.mark.parametrize("seed", range(6))
def test_cone_grad_random_vs_psr(Q, eng, oracle_mod, seed):
    rng = np.random.default_rng([31, seed])
    n = int(rng.integers(4, 15))
    kinds = (W.RX, W.RY, W.RZ, W.CZ, W.CNOT) if seed % 3 else (W.RX, W.RY, W.RZ, W.CZ, W.CNOT, W.U1)
    c = W.random_circuit(n, 60, rng, kinds=kinds, p_fixed=0.1)
    th = W.angles(max(c.n_params, 1), [31, seed])[: c.n_params]
    letters = "Z" if seed % 2 == 0 else "XYZ"
    H = W.random_hamiltonian(n, 10, rng, max_weight=min(n, 3), letters=letters)
    mode = Q.MODE_LIGHTCONE if seed % 4 == 1 else Q.MODE_LIGHTCONE_FACTORED
    say("cone grad random", seed, n, c.n_params, "mode", mode)
    psr = oracle_mod.grad_psr(c, H, th)
    E, g = eng.expect_grad(c, H, th, mode=mode)
    assert abs(E - oracle_mod.expect(c, H, th)) <= tol(H, 0)
    np.testing.assert_allclose(g, psr, atol=tol(H, 0))


def test_cone_grad_c128(Q, eng, oracle_mod):
    rng = np.random.default_rng([32, 0])
    c = W.brickwork_ry_rz_cnot(11, 3)
    H = W.tfim(11, 0.6)
    th = W.angles(c.n_params, [32, 1])
    say("cone grad c128")
    for mode in (Q.MODE_LIGHTCONE, Q.MODE_LIGHTCONE_FACTORED):
        E, g = eng.expect_grad(c, H, th, mode=mode, dtype=Q.C128)
        assert abs(E - oracle_mod.expect(c, H, th)) <= tol(H, 1)
        np.testing.assert_allclose(g, oracle_mod.grad_psr(c, H, th), atol=tol(H, 1))
    del rng


def test_cone_grad_n500_vs_oracle(Q, eng, oracle_mod):
    """n=500, 4 layers of RY + CZ brickwork, 3-regular MaxCut: E and sampled gradient entries."""
    w = W.lightcone_maxcut()
    idx = np.array([0, 1, 250, 499, 500, 1001, 1500, 1999], dtype=np.int32)
    want_E, _ = oracle_mod.expect_lightcone(w.circuit, w.H, w.theta)
    want_g = oracle_mod.grad_psr_lightcone(w.circuit, w.H, w.theta, idx)
    for mode in (Q.MODE_LIGHTCONE_FACTORED, Q.MODE_LIGHTCONE):
        say("cone grad n500 mode", mode)
        E, g = eng.expect_grad(w.circuit, w.H, w.theta, mode=mode)
        assert abs(E - want_E) <= tol(w.H, 0), (E, want_E)
        np.testing.assert_allclose(g[idx], want_g, atol=tol(w.H, 0))
        assert np.all(np.isfinite(g))


def test_cone_grad_product_state_n500(Q, eng):
    """One RY layer: d<H>/dt_i = -sin t_i sum over neighbours j of cos t_j."""
    n = 500
    b = W.GateListBuilder(n)
    for q in range(n):
        b.rot(W.RY, q)
    c = b.build()
    edges = W.random_regular3(n, np.random.default_rng([3, 0]))
    H = W.maxcut(edges)
    th = W.angles(n, [3, 500, 7])
    say("cone grad product n500")
    E, g = eng.expect_grad(c, H, th, mode=Q.MODE_LIGHTCONE_FACTORED)
    cs = np.cos(th)
    want = np.zeros(n)
    for a, bb in edges:
        want[a] += -math.sin(th[a]) * cs[bb]
        want[bb] += -math.sin(th[bb]) * cs[a]
    np.testing.assert_allclose(g, want, atol=tol(H, 0))
    assert abs(E - sum(cs[a] * cs[bb] for a, bb in edges)) <= tol(H, 0)


def test_cone_grad_equals_dense_grad(Q, eng):
    """The same gradient two ways on the device: full-state adjoint and per-cone adjoint."""
    w = W.batched_grad_tfim(batch=2, n=14, depth=3)
    say("cone grad vs dense n14")
    E0, g0 = eng.expect_grad(w.circuit, w.H, w.theta)
    for mode in (Q.MODE_LIGHTCONE, Q.MODE_LIGHTCONE_FACTORED):
        E1, g1 = eng.expect_grad(w.circuit, w.H, w.theta, mode=mode)
        np.testing.assert_allclose(E1, E0, atol=2 * tol(w.H, 0))
        np.testing.assert_allclose(g1, g0, atol=2 * tol(w.H, 0))
    # the same plan on the same input gives the same bits
    E2, g2 = eng.expect_grad(w.circuit, w.H, w.theta, mode=Q.MODE_LIGHTCONE_FACTORED)
    np.testing.assert_array_equal(E2, E1)
    np.testing.assert_array_equal(g2, g1)


def test_cone_grad_autograd(Q, eng, oracle_mod):
    import torch

    from paper_2112_10239_amd.autograd import expectation_cones

    c = W.brickwork_ry_cz(40, 3)
    H = W.maxcut(W.random_regular3(40, np.random.default_rng([33, 40])))
    th = W.angles(c.n_params, [33, 1])
    theta = torch.tensor(th[None, :], dtype=torch.float64, device="cuda:0", requires_grad=True)
    say("cone autograd n40")
    E = expectation_cones(theta, eng, c, H)
    (2.0 * E.sum()).backward()
    idx = np.array([0, 39, 40, 80, 119], dtype=np.int32)
    want = oracle_mod.grad_psr_lightcone(c, H, th, idx)
    np.testing.assert_allclose(theta.grad[0].cpu().numpy()[idx], 2.0 * want, atol=2 * tol(H, 0))
    want_E, _ = oracle_mod.expect_lightcone(c, H, th)
    assert abs(float(E[0]) - want_E) <= tol(H, 0)


def test_cone_grad_errors(Q, eng):
    w = W.lightcone_maxcut(n=60, depth=2)
    with pytest.raises(Q.QsimError):
        eng.expect_grad(w.circuit, w.H, w.theta, mode=99)
    small = Q.Context(0, cone_cap=4)
    try:
        with pytest.raises(Q.QsimError) as ei:
            small.expect_grad(w.circuit, w.H, w.theta, mode=Q.MODE_LIGHTCONE)
        assert ei.value.code == Q.qsim.ETOOBIG
    finally:
        small.close()


# --- reduced density matrices (partial trace on the matrix cores) --------------------------

def _state(Q, eng, c, th, dtype=0, batch=1):
    st = eng.create_state(c.n, batch=batch, dtype=dtype)
    st.apply_layer(c.gates, np.tile(th, (batch, 1)) if c.n_params else None, c.n_params, c.mats)
    return st


@pytest.mark.parametrize("keep", [[0], [1, 0], [0, 1, 2, 3, 4, 5, 6], [9, 2, 5], [3, 11, 0, 7, 6],
                                  list(range(12))])
def test_density_small_vs_oracle(Q, eng, oracle_mod, keep):
    w = W.dense_tfim(n=12, depth=3)
    say("density n12 keep", keep)
    st = _state(Q, eng, w.circuit, w.theta)
    rho = st.reduced_density(keep)[0]
    psi_gpu = st.to_host()[0]
    st.destroy()
    # the kernel's arithmetic against the oracle on the same (device) state
    np.testing.assert_allclose(rho, oracle_mod.partial_trace(psi_gpu, 12, keep), atol=2e-6)
    # end to end against the oracle's own state
    psi = oracle_mod.statevector(w.circuit, w.theta)
    np.testing.assert_allclose(rho, oracle_mod.partial_trace(psi, 12, keep), atol=1e-5)
    np.testing.assert_array_equal(rho, rho.conj().T)


def test_density_c128_batch(Q, eng, oracle_mod):
    w = W.batched_grad_tfim(batch=2, n=10, depth=3)
    say("density c128 batch 2")
    st = eng.create_state(10, batch=2, dtype=Q.C128)
    st.apply_layer(w.circuit.gates, w.theta, w.circuit.n_params, w.circuit.mats)
    keep = [4, 0, 8, 2]
    rho = st.reduced_density(keep)
    st.destroy()
    for b in range(2):
        psi = oracle_mod.statevector(w.circuit, w.theta[b])
        np.testing.assert_allclose(rho[b], oracle_mod.partial_trace(psi, 10, keep), atol=1e-12)


@pytest.mark.parametrize("m", [10, 14])
def test_density_n20_paper_sizes(Q, eng, m):
    """n=20 keeping 10 or 14 qubits: sampled entries against direct sums on the same state,
    trace 1, exact Hermitian symmetry, and <Z_q> of kept qubits equal to the state's."""
    import torch

    w = W.dense_tfim(n=20, depth=4)
    say("density n20 m", m)
    st = _state(Q, eng, w.circuit, w.theta)
    keep = list(range(m))
    N = 1 << m
    rho_t = torch.empty((N, N), dtype=torch.complex64, device="cuda:0")
    st.reduced_density(keep, out=rho_t)
    psi = st.to_host()[0].astype(np.complex128)
    zq = st.expect(W.Hamiltonian.from_terms([(1.0, [(3, "Z")])]))[0]
    st.destroy()
    rho = rho_t.cpu().numpy()
    M = psi.reshape(1 << (20 - m), N)  # row k, column i (kept qubits are the low bits)
    rng = np.random.default_rng([42, m])
    for _ in range(64):
        i, j = (int(x) for x in rng.integers(0, N, size=2))
        want = np.dot(M[:, i], np.conj(M[:, j]))
        assert abs(rho[i, j] - want) <= 2e-6, (i, j, rho[i, j], want)
    diag = np.real(np.diag(rho)).astype(np.float64)
    assert abs(diag.sum() - 1.0) <= 1e-4
    sign = 1.0 - 2.0 * ((np.arange(N) >> 3) & 1)
    assert abs(float(np.dot(diag, sign)) - zq) <= 1e-5
    i = rng.integers(0, N, size=256)
    j = rng.integers(0, N, size=256)
    np.testing.assert_array_equal(rho[i, j], np.conj(rho[j, i]))


def test_density_errors(Q, eng):
    st = eng.create_state(6)
    try:
        for bad in ([0, 0], [6], [-1], []):
            with pytest.raises(Q.QsimError):
                st.reduced_density(bad)
    finally:
        st.destroy()


@pytest.mark.parametrize("n,depth", [(16, 2), (20, 3), (22, 4)])
def test_lightcone_factored_groups_vs_oracle(Q, eng, oracle_mod, n, depth):
    """RY+RZ+CNOT brickwork cones: rotation runs on register bits become factored
    groups and CNOT runs exit permutations inside the cones; cones above 13 qubits
    (n = 22, depth 4) keep their state in scratch between passes."""
    say("lightcone factored groups", n, depth)
    c = W.brickwork_ry_rz_cnot(n, depth)
    H = W.tfim(n, 0.7)
    th = W.angles(c.n_params, [33, n, depth])
    want = oracle_mod.expect(c, H, th)
    for mode in (Q.MODE_LIGHTCONE, Q.MODE_LIGHTCONE_FACTORED):
        got = eng.expect_circuit(c, H, th, mode=mode)
        assert abs(got - want) <= tol(H, 0), (mode, got, want)
    # term by term (the cone of each term against the oracle's full state)
    _, ref, _ = oracle_mod.expect_state(n, oracle_mod.statevector(c, th), H)
    for mode in (Q.MODE_LIGHTCONE, Q.MODE_LIGHTCONE_FACTORED):
        np.testing.assert_allclose(eng.expect_terms(c, H, th, mode=mode), ref, atol=TOL64, err_msg=f"mode {mode}")
