"""Shared comparison helper of the GPU parity tests."""
import sys

import numpy as np


def assert_rows_close(a, b, n_gel, rel):
    """|a - b| <= rel * (largest |b| entry of the same row block): the gel
    rows and the indenter rows (k_t = 1e8 N/m, orders stiffer) are separate
    blocks, so the gel rows are not checked against the indenter's scale."""
    for sl, name in ((slice(0, n_gel), "gel"), (slice(n_gel, None), "indenter")):
        scale = np.abs(b[sl]).max() if b[sl].size else 0.0
        d = np.abs(a[sl] - b[sl]).max() if b[sl].size else 0.0
        print(f"    {name} rows: max |diff| {d:.3e}, scale {scale:.3e}", flush=True)
        sys.stdout.flush()
        assert (d <= rel * scale) if scale > 0 else d == 0.0, (name, d, scale)
