"""GPU checks of the dense five-qubit block (qsim_apply_block5) on the matrix
cores and on the vector ALUs, through the C-ABI.

The block is a 32 x 32 unitary formed in the test from a random gate list on
qubits 0..4 (every gate kind: RX/RY/RZ at random angles, U1, CNOT, CZ in both
directions), an input, not a computed result.  The expected state is the
oracle's: the preparation circuit followed by the same gate list, run gate by
gate in complex128.  The kernel rounds the block once to fp32 and sums 32
products per output, so each complex64 amplitude is compared at 2e-5.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL = 2e-5


@pytest.fixture(scope="module")
def Q():
    import paper_2112_10239_amd as Q

    return Q


@pytest.fixture(scope="module")
def eng(Q):
    ctx = Q.Context(0)
    yield ctx
    ctx.close()


def say(*a):
    print(*a, flush=True)


def _one_qubit(kind, t, mat):
    c, s = math.cos(t / 2), math.sin(t / 2)
    if kind == W.RX:
        return np.array([[c, -1j * s], [-1j * s, c]])
    if kind == W.RY:
        return np.array([[c, -s], [s, c]])
    if kind == W.RZ:
        return np.array([[c - 1j * s, 0], [0, c + 1j * s]])
    return np.asarray(mat, dtype=np.complex128).reshape(2, 2)


def block_unitary(c, theta):
    """The 32 x 32 matrix of a gate list on qubits 0..4 (index bit q = qubit q): the
    product of every gate's matrix in application order."""
    U = np.eye(32, dtype=np.complex128)
    for g, row in enumerate(c.gates):
        k, q0, q1 = int(row["kind"]), int(row["q0"]), int(row["q1"])
        M = np.zeros((32, 32), dtype=np.complex128)
        if k in W.TWO_QUBIT:
            for i in range(32):
                if k == W.CNOT:
                    j = i ^ (1 << q1) if (i >> q0) & 1 else i
                    M[j, i] = 1
                else:
                    M[i, i] = -1 if ((i >> q0) & 1) and ((i >> q1) & 1) else 1
        else:
            t = float(theta[row["param"]]) if int(row["param"]) >= 0 else float(row["angle"])
            m = _one_qubit(k, t, c.mats.get(g))
            for i in range(32):
                for b in range(2):
                    j = (i & ~(1 << q0)) | (b << q0)
                    M[j, i] += m[b, (i >> q0) & 1]
        U = M @ U
    return U


def _concat(prep, blk):
    """prep then blk as one circuit on prep.n qubits (blk's parameters after prep's)."""
    b = W.GateListBuilder(prep.n)
    for c, off in ((prep, 0), (blk, prep.n_params)):
        for g, row in enumerate(c.gates):
            k = int(row["kind"])
            if k in W.TWO_QUBIT:
                b.two(k, int(row["q0"]), int(row["q1"]))
            elif k == W.U1:
                b.custom(int(row["q0"]), c.mats[g])
            elif int(row["param"]) >= 0:
                b.rows.append((k, int(row["q0"]), -1, off + int(row["param"]), 0.0))
                b.n_params = max(b.n_params, off + int(row["param"]) + 1)
            else:
                b.rot(k, int(row["q0"]), fixed_angle=float(row["angle"]))
    return b.build()


@pytest.mark.parametrize("n,batch", [(10, 1), (12, 1), (9, 2)])
def test_block5_both_methods_vs_oracle(Q, eng, oracle_mod, n, batch):
    rng = np.random.default_rng([71, n, batch])
    prep = W.random_circuit(n, 6 * n, rng)
    blk = W.random_circuit(5, 40, rng)
    full = _concat(prep, blk)
    # per-row preparation angles, one block (the same angles) for every row
    th_blk = W.angles(max(blk.n_params, 1), [71, n, 99])[: blk.n_params]
    th_prep = np.stack([W.angles(max(prep.n_params, 1), [71, n, b])[: prep.n_params] for b in range(batch)])
    U = block_unitary(blk, th_blk)
    for method in (0, 1):
        say("block5", n, batch, "method", method)
        st = eng.create_state(n, batch=batch, dtype=Q.C64)
        st.apply_layer(prep.gates, th_prep, prep.n_params, mats=prep.mats)
        ms = st.apply_block5(U, method)
        psi = st.to_host()
        st.destroy()
        assert ms > 0
        for b in range(batch):
            want = oracle_mod.statevector(full, np.concatenate([th_prep[b], th_blk]))
            err = np.abs(psi[b] - want).max()
            assert err <= TOL, (method, b, err)


def test_block5_methods_agree_and_errors(Q, eng):
    rng = np.random.default_rng(72)
    z = rng.normal(size=(32, 32)) + 1j * rng.normal(size=(32, 32))
    U, _ = np.linalg.qr(z)
    out = []
    for method in (0, 1):
        say("block5 agree", method)
        st = eng.create_state(11, batch=1, dtype=Q.C64)
        c = W.brickwork_ry_rz_cnot(11, 2)
        st.apply_layer(c.gates, W.angles(c.n_params, [72, 1])[None, :], c.n_params)
        st.apply_block5(U, method)
        st.apply_block5(U.conj().T, method)  # U^dagger U = I: back to the prepared state
        out.append(st.to_host()[0])
        st.destroy()
    ref = eng.create_state(11, batch=1, dtype=Q.C64)
    ref.apply_layer(c.gates, W.angles(c.n_params, [72, 1])[None, :], c.n_params)
    psi0 = ref.to_host()[0]
    ref.destroy()
    for o in out:
        assert np.abs(o - psi0).max() <= 2 * TOL
    with pytest.raises(Q.QsimError):  # complex128 states are not supported
        s = eng.create_state(8, batch=1, dtype=Q.C128)
        try:
            s.apply_block5(U, 0)
        finally:
            s.destroy()
    with pytest.raises(Q.QsimError):  # 2^(6-5) = 2 rows: not a multiple of 32 for the matrix cores
        s = eng.create_state(6, batch=1, dtype=Q.C64)
        try:
            s.apply_block5(U, 0)
        finally:
            s.destroy()
