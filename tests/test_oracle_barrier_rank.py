"""The unmollified pair barrier Hessian has rank at most five.

For a fixed distance type the squared distance is |sum_k c_k x_k|^2
minimised over at most two feature parameters, so its Hessian is
2 c c^T (x) I3 (rank 3) minus an envelope term of rank at most two, and the
distance gradient lies in the span of the first; the barrier Hessian
kappa (b'' grad d grad d^T + b' Hess d) lives in that span too. The GPU pair
kernel projects it to PSD there (a 5 x 5 eigenproblem instead of 12 x 12).
This pins the premise on the oracle's exact pair Hessian (itself pinned by
finite differences in test_oracle_distance.py) for every point-triangle and
edge-edge distance type: at most five eigenvalues above roundoff, and the
PSD projection computed in the span of the five leading eigenvectors equals
the oracle's projection of the whole 12 x 12."""
import numpy as np

import oracle as O

DHAT = 1e-4
KAPPA = 1e4
MM = 1e-3


def _check(kind, x):
    d = (O.pt_distance if kind == 0 else O.ee_distance)(x)[0]
    x = x * (0.5 * DHAT / d)  # the distance type does not depend on scale
    _, _, H = O.pair_barrier(kind, x, DHAT, KAPPA, 0.0, project=False)
    w, V = np.linalg.eigh(H)
    order = np.argsort(-np.abs(w))
    w, V = w[order], V[:, order]
    assert np.abs(w[5:]).max() <= 1e-9 * np.abs(w).max(), w
    _, _, Hp = O.pair_barrier(kind, x, DHAT, KAPPA, 0.0, project=True)
    Q = V[:, :5]
    m, U = np.linalg.eigh(Q.T @ H @ Q)
    P = Q @ U
    assert np.abs(Hp - (P * np.maximum(m, 0)) @ P.T).max() <= 1e-9 * np.abs(H).max()


def test_pair_hessian_rank_every_type():
    rng = np.random.default_rng(5)
    seen = {0: set(), 1: set()}
    tries = 0
    while (len(seen[0]) < 7 or len(seen[1]) < 9) and tries < 20000:
        tries += 1
        x = rng.uniform(-1, 1, 12) * MM
        if rng.random() < 0.3:  # toward the degenerate-feature types
            x[9:12] = x[6:9] + rng.uniform(-0.3, 0.3, 3) * MM
        for kind, fn in ((0, O.pt_distance), (1, O.ee_distance)):
            _, t = fn(x)
            if t not in seen[kind]:
                _check(kind, x)
                seen[kind].add(t)
    assert seen[0] == set(range(7)) and seen[1] == set(range(9))
