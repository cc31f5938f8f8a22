"""Write the stored expected values of the small configuration.

Calls only the oracle (and the seeded input generator for its input):
    python tests/golden/make_golden.py
Output: tests/golden/oracle_small_seed0.json
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2004_00923_amd.synth import gen_stack, sha256  # noqa: E402

LAM, PITCH, Z = 785e-9, 20e-6, 0.3
K_LO, K_HI = 2, 31
SAMPLES = [(0, 0), (64, 64), (10, 100), (127, 3), (70, 90), (40, 20)]


def main():
    frames = gen_stack(0, 32, 128, 128)
    r = oracle.pipeline_ref(frames, LAM, Z, PITCH, K_LO, K_HI)
    out = {
        "what": "32 x 128 x 128 stack, seed 0, lambda 785 nm, pitch 20 um, z 0.3 m, kept components 2..31",
        "writer": "tests/golden/make_golden.py (oracle only)",
        "stack_sha256": sha256(frames),
        "evals": [float(x) for x in r["evals"]],
        "cov_diag": [float(x) for x in np.diag(r["cov"]).real],
        "image_sum": float(r["image"].sum()),
        "image_max": float(r["image"].max()),
        "image_samples": [[y, x, float(r["image"][y, x])] for y, x in SAMPLES],
        "holo_samples": [[t, y, x, float(r["holo"][t, y, x].real), float(r["holo"][t, y, x].imag)]
                         for t, (y, x) in zip([0, 5, 31, 17, 9, 2], SAMPLES)],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_small_seed0.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
