"""Writes c2_seed0_final.txt: the FP64 oracle's positions after the full
50-step trajectory of the 40x50x8 gel / cylinder (seed 0) workload, sampled
at every 97th vertex, for the fixed-error check of the benchmarked
configuration (max over the samples of |x - x_oracle| / L).

Calls only the oracle. Takes about two hours on one core."""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2411_04776_amd import scenes as S  # noqa: E402


def main():
    sc = S.config2(0)
    o = O.OracleScene(sc, pcg_tol=1e-12)
    t0 = time.time()
    for k in range(1, sc.n_steps + 1):
        rc, st = o.step(sc.poses[k])
        print(f"step {k}: rc={rc} newton={st.newton_iters} ({time.time() - t0:.0f} s)", flush=True)
    x = o.x
    idx = np.arange(0, o.n, 97)
    with open(os.path.join(HERE, "c2_seed0_final.txt"), "w") as f:
        f.write("# FP64 oracle, config 2 seed 0 (40x50x8 gel, cylinder r=4.55 mm), positions after step 50\n")
        f.write(f"# written by tests/golden/make_c2_final.py; L = {sc.bbox_diag!r}\n")
        f.write("# vertex x y z (m)\n")
        for i in idx:
            f.write(f"{i} {float(x[i, 0])!r} {float(x[i, 1])!r} {float(x[i, 2])!r}\n")


if __name__ == "__main__":
    main()
