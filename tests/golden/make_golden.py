"""Writes the stored reference values under tests/golden/ from the FP64 oracle only.

small_fp64_ista_safe.txt: the small FP64 configuration (100 x 500 Gaussian dictionary,
Bernoulli(0.05)-Gaussian code, noise 0.01 N(0,1), lambda = 0.5 lambda_*), run by the
dynamic-screening algorithm (Algorithm 3 with the ISTA update of Table 1 and the SAFE
sphere test of Lemma 1, as in Algorithm 5) for exactly 500 iterations with L = ||D||_2^2.
The paper prints no numeric worked example, so these values come from the oracle; they
guard the configuration against unintended changes.

Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1412_4080_amd import datagen  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "small_fp64_ista_safe.txt")


def main():
    c = datagen.lasso_small_fp64()
    D, y = c["D"], c["y"]
    L = oracle.spectral_norm_sq(D)
    r = oracle.solve_lasso(D, y, lam_ratio=c["lam_ratio"], rule=c["rule"], test=c["test"], L=L,
                           max_iter=c["max_iter"], gap_tol=c["gap_tol"], record=True)
    lines = ["# small FP64 configuration: Algorithm 3, ISTA (Table 1), SAFE (Lemma 1), 500 iterations",
             "# written by tests/golden/make_golden.py from the FP64 oracle",
             f"lambda {r.lam!r}", f"lambda_max {r.lam_max!r}", f"L {L!r}", f"iters {r.iters}",
             f"primal_p {r.primal_p!r}", f"gap {r.gap!r}", f"r_min {r.r_min!r}",
             "n_active " + " ".join(str(h["n_active"]) for h in r.history),
             "nnz " + " ".join(str(h["nnz"]) for h in r.history)]
    for i in np.flatnonzero(r.x):
        lines.append(f"x {i} {float(r.x[i])!r}")
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
