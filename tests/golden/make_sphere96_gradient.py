"""Write sphere96_gradient_segment.json: the oracle's gradient of the first
checkpoint segment of the 96^3 adjoint workload.

Workload: frozen sphere r = 4 in [-5,5]^3 on 96^3 nodes, u0 ~ U[0.2,0.8]
inside (seed 0), logistic f, ETD2RK (Section 3.2) with h = 0.01, 8 steps
(the first segment of the 40-step run checkpointed every 8 steps), loss
L = sum over the unknowns of U_8^2.  The oracle (oracle.adjoint.gradient,
Krylov route self-converged to 1e-13) takes about 12 minutes here, too long
for the GPU test suite, so this script stores what the GPU test compares:
L, dL/dbeta, |dL/dU_0|, the projections of dL/dU_0 on 8 seeded Gaussian
vectors (numpy default_rng(100 + k)), and dL/dU_0 at 2048 unknowns drawn
with default_rng(7) (indices in the oracle's gather order, which is
lexicographic over the box, x fastest).

Usage (from the repository root): python tests/golden/make_sphere96_gradient.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.adjoint import gradient  # noqa: E402
from oracle.etd import logistic  # noqa: E402
from oracle.geometry import Grid  # noqa: E402
from oracle.operator import build_operator  # noqa: E402
from paper_2209_15095_amd import inputs  # noqa: E402

STEPS = 8
NSAMPLE = 2048
NPROJ = 8


def main():
    w = inputs.sphere96()
    g = Grid(w.grid.dim, tuple(w.grid.n), tuple(w.grid.lo), tuple(w.grid.hi))
    op = build_operator(g, w.rho0, w.beta)
    f, df = logistic(w.a, w.b)
    t0 = time.time()
    L, gU, db = gradient(op.A, w.beta, w.h, op.gather(w.u0), STEPS, f, df, method="krylov")
    secs = time.time() - t0
    idx = np.sort(np.random.default_rng(7).choice(op.n, NSAMPLE, replace=False))
    proj = [float(np.random.default_rng(100 + k).standard_normal(op.n) @ gU) for k in range(NPROJ)]
    out = {
        "workload": "sphere96", "steps": STEPS, "h": w.h, "beta": w.beta, "n_unknowns": int(op.n),
        "L": L, "dL_dbeta": db, "grad_norm": float(np.linalg.norm(gU)), "projections": proj,
        "sample_index": [int(i) for i in idx], "sample_grad": [float(x) for x in gU[idx]],
        "oracle_seconds": secs,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sphere96_gradient_segment.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"wrote {path}: L {L:.15e} dL/dbeta {db:.15e} ({secs:.0f} s)")


if __name__ == "__main__":
    main()
