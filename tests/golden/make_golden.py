"""Writes the stored expected values under tests/golden/ from the oracle alone.

small_binary_gmres50.json: plain GMRES(50), complex128, tol 1e-8, on the
64 x 64 binary-pixel problem of workloads.small_binary(0) (the small seeded
case whose oracle solve finishes in seconds): iteration count, the first 400
entries of the least-squares residual history ||b - A x_i|| / ||b|| and the
solution's 2-norm.  Run from the repository root:

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import fdfd, gmres  # noqa: E402


def small_binary_gmres50():
    inst = W.small_binary(0)
    A = fdfd.assemble_instance(inst)
    x, info = gmres.gmres(A, inst.b, restart=50, tol=1e-8, maxit=20000)
    return {
        "case": "workloads.small_binary(0): 64x64, dx 40 nm, wavelength 1550 nm, 10-cell PML",
        "solver": "oracle gmres.gmres, restart 50, tol 1e-8, complex128",
        "iters": int(info["iters"]),
        "history_first_400": [float(v) for v in info["history"][:400]],
        "x_norm": float(np.linalg.norm(x)),
    }


if __name__ == "__main__":
    out = os.path.join(HERE, "small_binary_gmres50.json")
    with open(out, "w") as f:
        json.dump(small_binary_gmres50(), f, indent=1)
    print("wrote", out)
