"""Reader of the hand-worked fixtures under tests/golden/ (test helper only)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def fw_blocked_f32_cases():
    """Cases of golden/fw_blocked_f32_hand.txt as a list of dicts with keys
    name, n, block, W (n x n float32: edges, 0 on the diagonal, +inf elsewhere)
    and D (the hand-derived result, same layout)."""
    cases, cur = [], None
    with open(os.path.join(GOLDEN, "fw_blocked_f32_hand.txt")) as f:
        for line in f:
            tok = line.split("#", 1)[0].split()
            if not tok:
                continue
            if tok[0] == "case":
                n, b = int(tok[2]), int(tok[3])
                cur = {"name": tok[1], "n": n, "block": b, "edges": [], "expect": []}
            elif tok[0] in ("edge", "expect"):
                cur[tok[0] if tok[0] == "expect" else "edges"].append(
                    (int(tok[1]), int(tok[2]), float.fromhex(tok[3])))
            elif tok[0] == "end":
                n = cur["n"]
                W = np.full((n, n), np.inf, dtype=np.float32)
                D = np.full((n, n), np.inf, dtype=np.float32)
                np.fill_diagonal(W, 0)
                np.fill_diagonal(D, 0)
                for i, j, w in cur["edges"]:
                    W[i, j] = np.float32(w)
                    assert float(W[i, j]) == w, "fixture weight is not a binary32 value"
                for i, j, w in cur["expect"]:
                    D[i, j] = np.float32(w)
                    assert float(D[i, j]) == w, "fixture value is not a binary32 value"
                cases.append({"name": cur["name"], "n": n, "block": cur["block"], "W": W, "D": D})
                cur = None
    return cases
