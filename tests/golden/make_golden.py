"""Writes tests/golden/exact_small.json from the exact-rational oracle only.

Run from the repository root:  python tests/golden/make_golden.py
The file holds X_k (as fraction strings) for small integer matrices, the
transpose start X_0 = A^T / (||A||_1 ||A||_inf) and the identity start
X_0 = I / Tr(A), depths 1..3 and nests 1..3 (Theorem of Sec. II-D).
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import exact as ex  # noqa: E402

MATS = {
    "spd3": [[4, 1, 0], [1, 3, 1], [0, 1, 2]],
    "nonsym3": [[5, 2, -1], [1, 4, 0], [2, -1, 6]],
    "nonsym4": [[2, 1, 0, 0], [0, 3, 1, 0], [1, 0, 4, 1], [0, 1, 0, 5]],
}


def main():
    out = {"source": "oracle.exact (rational arithmetic); Theorem of Sec. II-D", "cases": []}
    for name, A in MATS.items():
        F = ex.to_frac(A)
        starts = {"transpose": ex.x0_transpose(F)}
        if name.startswith("spd"):
            starts["identity"] = ex.x0_scaled_identity(F)
        for kind, X0 in starts.items():
            for d in (1, 2, 3):
                X = X0
                for k in (1, 2, 3):
                    X = ex.nn_step_right(F, X, d)
                    out["cases"].append({"name": name, "A": A, "x0": kind, "d": d, "k": k,
                                         "X": [[str(v) for v in r] for r in X]})
    with open(os.path.join(HERE, "exact_small.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
