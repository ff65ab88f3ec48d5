"""Writes tests/golden/*.json from the CPU oracle only (no GPU path involved).

The paper prints no worked example with values, so these fixtures are the
oracle's complex128 results on the small seeded workloads; the oracle itself is
pinned by tests/test_oracle_pins.py.  Regenerate with:

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def main():
    oracle.build(force=False)
    w = W.small_ring_maxcut()
    E = oracle.expect(w.circuit, w.H, w.theta)
    _, terms = oracle.expect_lightcone(w.circuit, w.H, w.theta)
    g = oracle.grad_psr(w.circuit, w.H, w.theta)
    out = {"workload": w.name, "source": "oracle complex128 (oracle/qsim_oracle.c)",
           "edges": w.edges.tolist(), "E": E, "term_values": terms.tolist(), "grad_psr": g.tolist()}
    with open(os.path.join(HERE, "ring_maxcut_n10_d4.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("E =", E)


if __name__ == "__main__":
    main()
