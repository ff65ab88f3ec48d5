"""Host replay of dense plans against the oracle (no device use).

qsim_plan_trace lists what every stage of a dense plan applies, in order and on
index bits: fused single-qubit gates (their source gates), CNOTs and CZs of the
stage permutations (among them the index-bit swaps with which a relabelling
pass hands its low index bits to the next pass), and the Pauli terms, measured
where the plan measures them (X/Y terms as soon as every gate they do not
commute with has been applied).  The replay rebuilds that sequence as a circuit
on index bits, runs every prefix that ends at a term through
oracle.statevector and measures the term there with oracle.expect_state; the
weighted sum must equal oracle.expect of the original circuit.  A term measured
too early, a swap applied before a term it moves, or a term mapped to the wrong
index bit changes the sum.
"""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def Q():
    import paper_2112_10239_amd as Q

    return Q


def _pauli_ops(fmask: int, zmask: int):
    ops = []
    for b in range(64):
        f, z = (fmask >> b) & 1, (zmask >> b) & 1
        if f or z:
            ops.append((b, "Y" if f and z else "X" if f else "Z"))
    return ops


def replay(oracle_mod, c, H, th, rec, coef, srcs):
    """Sum of the traced term measurements (plus the identity part of H)."""
    rows, mats = [], {}
    E = sum(cf for cf, ops in H.terms() if not ops)
    n_terms = 0
    for r, w in zip(rec, coef):
        kind = int(r[0])
        if kind in (0, 5):
            for s in srcs[r[3]:r[3] + r[4]]:
                g = c.gates[int(s)]
                q = int(g["q0"]) if kind == 5 else int(r[1])
                if int(s) in c.mats:
                    mats[len(rows)] = c.mats[int(s)]
                rows.append((g["kind"], q, -1, g["param"], g["angle"]))
        elif kind == 1:
            rows.append((W.CNOT, int(r[2]), int(r[1]), -1, 0.0))
        elif kind == 2:
            rows.append((W.CZ, int(r[1]), int(r[2]), -1, 0.0))
        elif kind == 3:
            prefix = W.Circuit(c.n, np.array(rows, dtype=W.GATE_DTYPE), c.n_params, dict(mats))
            psi = oracle_mod.statevector(prefix, th)
            term = W.Hamiltonian.from_terms([(float(w), _pauli_ops(int(r[6]), int(r[7])))])
            E += oracle_mod.expect_state(c.n, psi, term)[0]
            n_terms += 1
        else:
            assert kind == 4, kind
    final = W.Circuit(c.n, np.array(rows, dtype=W.GATE_DTYPE), c.n_params, dict(mats))
    return E, n_terms, final


def _check(Q, oracle_mod, ctx, c, H, th, keep=False, dtype=None):
    rec, coef, srcs = ctx.plan_trace(c, H, keep=keep, dtype=Q.qsim.C64 if dtype is None else dtype)
    got, n_terms, final = replay(oracle_mod, c, H, th, rec, coef, srcs)
    assert n_terms == sum(1 for _, ops in H.terms() if ops)
    want = oracle_mod.expect(c, H, th)
    assert abs(got - want) <= 1e-9 * max(1.0, H.abs_coeff_sum()), (got, want)
    if keep:
        # a kept state ends with every qubit at its own index bit
        np.testing.assert_allclose(oracle_mod.statevector(final, th), oracle_mod.statevector(c, th), atol=1e-12)
    return rec


@pytest.mark.parametrize("n,depth", [(15, 3), (15, 7), (16, 5)])
@pytest.mark.parametrize("clow", [4, 5, 6])
def test_replay_tfim_relabelled(Q, oracle_mod, n, depth, clow):
    """Tiles of 2^12 amplitudes: several passes, relabelled, X terms early."""
    c = W.brickwork_ry_rz_cnot(n, depth)
    H = W.tfim(n, 0.7)
    th = W.angles(c.n_params, [60, n, depth])
    ctx = Q.Context(-1, tile_qubits=12, coalesce_bits=clow)
    try:
        rec = _check(Q, oracle_mod, ctx, c, H, th)
        ends = int((rec[:, 0] == 4).sum())
        assert ends > 3
    finally:
        ctx.close()


@pytest.mark.parametrize("off", [0, "OFF_RELABEL", "OFF_EARLY_TERMS", "OFF_PRODUCT", "OFF_ABSORB", "OFF_EXIT"])
@pytest.mark.parametrize("keep", [False, True])
def test_replay_switches(Q, oracle_mod, off, keep):
    import paper_2112_10239_amd.qsim as qs

    n, depth = 15, 6
    c = W.brickwork_ry_rz_cnot(n, depth)
    H = W.Hamiltonian.from_terms(list(W.tfim(n, 0.5).terms()) + [(0.3, [(1, "Y"), (3, "X")]), (0.25, [])])
    th = W.angles(c.n_params, [61, n])
    ctx = Q.Context(-1, tile_qubits=12, disable=getattr(qs, off) if off else 0)
    try:
        _check(Q, oracle_mod, ctx, c, H, th, keep=keep)
    finally:
        ctx.close()


@pytest.mark.parametrize("n,depth", [(14, 6), (15, 4), (16, 8)])
def test_replay_kept_state_relabelled(Q, oracle_mod, n, depth):
    """Kept final states relabel too: the last pass, or a pass of its own, puts every qubit
    back at its own index bit (checked on the replayed final state)."""
    import paper_2112_10239_amd.qsim as qs

    c = W.brickwork_ry_rz_cnot(n, depth)
    H = W.tfim(n, 0.6)
    th = W.angles(c.n_params, [64, n, depth])
    passes = {}
    for off in (0, qs.OFF_RELABEL):
        ctx = Q.Context(-1, tile_qubits=12, disable=off)
        try:
            rec = _check(Q, oracle_mod, ctx, c, H, th, keep=True)
            passes[off] = len(ctx.plan_passes(c, H, keep=True))
        finally:
            ctx.close()
    assert passes[0] <= passes[qs.OFF_RELABEL], passes


def test_replay_complex128(Q, oracle_mod):
    """complex128 plans (2^13-amplitude tiles, rotations one by one) relabel and measure early too."""
    n, depth = 16, 5
    c = W.brickwork_ry_rz_cnot(n, depth)
    H = W.tfim(n, 0.9)
    th = W.angles(c.n_params, [63, n])
    ctx = Q.Context(-1)
    try:
        _check(Q, oracle_mod, ctx, c, H, th, dtype=Q.qsim.C128)
    finally:
        ctx.close()


@pytest.mark.parametrize("seed", range(4))
def test_replay_random(Q, oracle_mod, seed):
    """Random gates (RX, RY, RZ, CZ, CNOT) and random Pauli strings up to weight 3."""
    rng = np.random.default_rng([62, seed])
    n = 14 + seed % 3
    c = W.random_circuit(n, 160, rng, kinds=(W.RX, W.RY, W.RZ, W.CZ, W.CNOT))
    H = W.random_hamiltonian(n, 12, rng, max_weight=3)
    th = W.angles(max(c.n_params, 1), [62, seed, 1])[: c.n_params]
    ctx = Q.Context(-1, tile_qubits=12)
    try:
        _check(Q, oracle_mod, ctx, c, H, th)
    finally:
        ctx.close()
