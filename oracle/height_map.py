"""Height map of a deformed gel surface -- test infrastructure only (the
oracle side of the library's ipc_height_map; only tests, the smoke check and
the benchmark's CPU leg use it).

The optical tactile renderers the paper pairs with the soft-body gel take a
height map of the sensing surface. Definition used here: for the pixel centre
(x0 + i dx, y0 + j dy), the indentation depth z_ref - z*, with z* the largest
height at which the vertical line through the centre meets an upward-facing
surface triangle (positive signed xy area, the triangles being oriented
outward); 0 where it meets none. Such a triangle contains the centre when its
three edge functions are all >= 0; z is the barycentric interpolation of the
vertex heights. Written straight
from that definition: every triangle against the pixels of its bounding box
(widened by two pixels), plain FP64 numpy.
"""
import numpy as np


def height_map(x, tris, x0, y0, dx, dy, nx, ny, z_ref):
    """x: (n, 3) positions; tris: (m, 3) vertex ids of the surface triangles
    to rasterise. Returns the (ny, nx) depth map."""
    x = np.asarray(x, dtype=np.float64)
    best = np.full((ny, nx), -np.inf)
    hit = np.zeros((ny, nx), dtype=bool)
    for t in np.asarray(tris):
        a, b, c = x[t[0]], x[t[1]], x[t[2]]
        area = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])
        if not area > 0.0:
            continue
        i0 = max(int(np.floor((min(a[0], b[0], c[0]) - x0) / dx)) - 2, 0)
        i1 = min(int(np.ceil((max(a[0], b[0], c[0]) - x0) / dx)) + 2, nx - 1)
        j0 = max(int(np.floor((min(a[1], b[1], c[1]) - y0) / dy)) - 2, 0)
        j1 = min(int(np.ceil((max(a[1], b[1], c[1]) - y0) / dy)) + 2, ny - 1)
        if i1 < i0 or j1 < j0:
            continue
        ii = np.arange(i0, i1 + 1)
        jj = np.arange(j0, j1 + 1)
        px = x0 + ii * dx
        py = y0 + jj * dy
        PX, PY = np.meshgrid(px, py)
        w0 = (c[0] - b[0]) * (PY - b[1]) - (c[1] - b[1]) * (PX - b[0])
        w1 = (a[0] - c[0]) * (PY - c[1]) - (a[1] - c[1]) * (PX - c[0])
        w2 = (b[0] - a[0]) * (PY - a[1]) - (b[1] - a[1]) * (PX - a[0])
        inside = (w0 >= 0) & (w1 >= 0) & (w2 >= 0)
        z = (w0 * a[2] + w1 * b[2] + w2 * c[2]) / area
        sub = best[j0:j1 + 1, i0:i1 + 1]
        upd = inside & (z > sub)
        sub[upd] = z[upd]
        hit[j0:j1 + 1, i0:i1 + 1] |= inside
    out = np.zeros((ny, nx))
    out[hit] = z_ref - best[hit]
    return out
