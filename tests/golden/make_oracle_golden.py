"""Write the oracle's expected values for the full-size benchmark workloads.

Calls only the CPU oracle (``oracle/``) and the seeded input generators
(``workloads``); nothing here touches the HIP library.  Run from the repository root:

    python tests/golden/make_oracle_golden.py brick26      # ~4 min, one core
    python tests/golden/make_oracle_golden.py qaoa24 0     # one parameter set, ~15 min
    python tests/golden/make_oracle_golden.py merge-qaoa24 # join the per-set files

Files written:

* ``brick26_depth4.json``: the random brick circuit (section 7's random-circuit benchmark,
  in the seeded form the 30-qubit benchmark uses) at 26 qubits and depth 4, from |0...0>:
  2048 amplitudes at seeded indices plus the first and the last, <Z_q> for every qubit
  and <sum_q Z_q>.
* ``qaoa24_p8_sets.json``: the 24-qubit p = 8 QAOA MaxCut workload (section 7's QAOA
  benchmark, layer convention of section 6.2), energies and adjoint gradients of four of
  its 64 parameter sets.
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import statevector as O  # noqa: E402

BRICK = dict(n_qubits=26, depth=4, seed=2406, samples=2048, sample_seed=26)
QAOA_SETS = (0, 21, 42, 63)


def brick26():
    n, depth = BRICK["n_qubits"], BRICK["depth"]
    circ, H = W.brick_workload(n, depth, BRICK["seed"])
    psi = O.simulate(circ)
    rng = np.random.default_rng(BRICK["sample_seed"])
    idx = np.concatenate([[0, 2 ** n - 1], rng.integers(0, 2 ** n, BRICK["samples"])]).astype(np.int64)
    zq = [float(O.expectation(psi, n, [(1.0, ((q, "Z"),))]).real) for q in range(n)]
    out = {
        "citation": "Section 7 (random-circuit benchmark), seeded brick form: per layer a Haar 2x2 unitary on "
                    "every qubit, then CZ on (2i, 2i+1) for even layers and (2i+1, 2i+2) for odd layers.",
        "written_by": "tests/golden/make_oracle_golden.py brick26 (CPU oracle only)",
        **{k: BRICK[k] for k in ("n_qubits", "depth", "seed", "sample_seed")},
        "index": idx.tolist(),
        "re": [float(v) for v in psi[idx].real],
        "im": [float(v) for v in psi[idx].imag],
        "norm": float(np.vdot(psi, psi).real),
        "z": zq,
        "sum_z": float(O.expectation(psi, n, H).real),
    }
    with open(os.path.join(HERE, "brick26_depth4.json"), "w") as f:
        json.dump(out, f, indent=1)


def qaoa24_set(b):
    circ, H, params, edges = W.qaoa_workload()
    E, g = O.grad_adjoint(circ, H, params[b])
    with open(os.path.join(HERE, f"_qaoa24_set{b}.json"), "w") as f:
        json.dump({"set": b, "params": params[b].tolist(), "energy": float(E), "grad": g.tolist()}, f)


def merge_qaoa24():
    _, _, _, edges = W.qaoa_workload()
    sets = []
    for b in QAOA_SETS:
        p = os.path.join(HERE, f"_qaoa24_set{b}.json")
        with open(p) as f:
            sets.append(json.load(f))
    out = {
        "citation": "Section 7 (QAOA benchmark, adjoint-method gradients) with the layer convention of "
                    "section 6.2: start |+>^24, per layer prod_edges exp(-i gamma Z_i Z_j) then RX(beta) on "
                    "every qubit; H = sum_edges (1 - Z_i Z_j) / 2; parameters [gamma_1..8, beta_1..8].",
        "written_by": "tests/golden/make_oracle_golden.py qaoa24 / merge-qaoa24 (CPU oracle only)",
        "n_qubits": 24, "p": 8, "edges": [list(e) for e in edges],
        "sets": sets,
    }
    with open(os.path.join(HERE, "qaoa24_p8_sets.json"), "w") as f:
        json.dump(out, f, indent=1)
    for b in QAOA_SETS:
        os.remove(os.path.join(HERE, f"_qaoa24_set{b}.json"))


if __name__ == "__main__":
    what = sys.argv[1]
    if what == "brick26":
        brick26()
    elif what == "qaoa24":
        qaoa24_set(int(sys.argv[2]))
    elif what == "merge-qaoa24":
        merge_qaoa24()
    else:
        raise SystemExit(f"unknown target {what!r}")
