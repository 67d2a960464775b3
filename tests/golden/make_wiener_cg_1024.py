"""Write tests/golden/wiener_cg_1024.txt: the Wiener filter (Eq. 2-3) of the
paper-size recipe scaled to 1024 x 1024 (data seed 0), solved by the oracle's
conjugate-gradient route (oracle.messenger.wiener_cg, pinned against the dense
solve of Eq. 2), at 2048 pixels drawn by a seeded generator, plus the L2 norm
of the whole solution.  Only the oracle and the input generator are called.

    python tests/golden/make_wiener_cg_1024.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import messenger as om  # noqa: E402
from paper_1810_02821_amd import synth  # noqa: E402

N, SEED, N_PIX, TOL = 1024, 0, 2048, 1e-10


def main():
    prob = synth.config_128(SEED, N)
    s, iters = om.wiener_cg(prob, tol=TOL)
    res = om.residual(prob, s)
    idx = np.sort(np.random.default_rng(12345).choice(N * N, size=N_PIX, replace=False))
    out = os.path.join(HERE, "wiener_cg_1024.txt")
    with open(out, "w") as f:
        f.write(f"# config_128 recipe, size {N}, data seed {SEED}: Wiener filter by oracle.messenger.wiener_cg\n")
        f.write(f"# cg tol {TOL:g}, {iters} iterations, residual of the normal equations {res:.3e}\n")
        f.write(f"# norm {np.linalg.norm(s):.17e}\n")
        f.write("# flat row-major pixel index, value\n")
        for i in idx:
            f.write(f"{i} {s.flat[i]:.17e}\n")
    print(out, iters, res)


if __name__ == "__main__":
    main()
