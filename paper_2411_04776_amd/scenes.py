"""Seeded synthetic scenes for the gel-pad IPC step: meshes, indenter shapes and
per-step indenter poses.

This module is pure input generation. It holds none of the solver's arithmetic
(no elasticity, distances, barrier, CCD or linear algebra), so both the CPU
oracle and the HIP path may consume its output as data.

The paper's GIPC pipeline (section "General GIPC Simulation Pipeline") creates
each soft object from a tetrahedral mesh and drives kinematic vertices by target
values each frame (section "GIPC Attachments"). The scenes below stand in for its
Isaac Sim assets: a GelSight-Mini-sized box gel meshed as a structured grid with a
Kuhn 6-tet split per hex, and a rigid indenter (icosphere, cylinder, box edge or
bumpy heightfield plate) whose vertices are pulled to a rigid pose per step.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Gel pad size in metres (x, y, z); origin at the bottom corner, z up.
GEL_SIZE = (0.020, 0.025, 0.004)

# Material and contact constants shared by every workload.
E_YOUNG = 0.3e6
NU = 0.45
RHO = 1000.0
DHAT = 1e-4
KAPPA = 1e4
K_TARGET = 1e8


# ----------------------------------------------------------------------------
# Gel: structured grid, Kuhn split
# ----------------------------------------------------------------------------

# Axis permutations in the order xyz, xzy, yxz, yzx, zxy, zyx and their parity.
_KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))
_KUHN_ODD = (False, True, True, False, False, True)


def grid_gel(nx: int, ny: int, nz: int, size=GEL_SIZE):
    """Vertex grid nx*ny*nz over the box `size`, each hex split into 6 tets.

    Vertex id = i + nx*(j + ny*k), x fastest, z up. Each hex walks the six
    monotone paths from its (0,0,0) corner to its (1,1,1) corner; odd paths swap
    their 2nd and 3rd vertex so every tet is positively oriented.
    Returns X (n,3) float64, T (m,4) int32, fixed (n,) uint8 (bottom face = 1).
    """
    if nx < 2 or ny < 2 or nz < 2:
        raise ValueError("grid needs at least 2 vertices per axis")
    xs = np.linspace(0.0, size[0], nx)
    ys = np.linspace(0.0, size[1], ny)
    zs = np.linspace(0.0, size[2], nz)
    K, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X = np.stack([xs[I.ravel()], ys[J.ravel()], zs[K.ravel()]], axis=1).astype(np.float64)
    fixed = (K.ravel() == 0).astype(np.uint8)

    hi, hj, hk = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), np.arange(nz - 1), indexing="ij")
    hi = hi.transpose(2, 1, 0).ravel()
    hj = hj.transpose(2, 1, 0).ravel()
    hk = hk.transpose(2, 1, 0).ravel()
    step = (1, nx, nx * ny)
    c000 = hi + nx * (hj + ny * hk)
    c111 = c000 + step[0] + step[1] + step[2]
    tets = []
    for perm, odd in zip(_KUHN_PERMS, _KUHN_ODD):
        a, b, _ = perm
        v0 = c000
        v1 = v0 + step[a]
        v2 = v1 + step[b]
        v3 = c111
        if odd:
            v1, v2 = v2, v1
        tets.append(np.stack([v0, v1, v2, v3], axis=1))
    # hex-major order: the 6 tets of one hex are consecutive
    T = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    return X, T, fixed


def soft_ball(n: int, radius: float, center):
    """Tet mesh of a ball: the n^3 Kuhn grid of the cube [-r, r]^3 mapped
    radially onto the ball, p -> p |p|_inf / |p|_2 (cube surface onto the
    sphere; the map scales each ray by a positive factor constant along it, so
    its Jacobian determinant is that factor cubed and no tet turns over).
    Returns X (n^3, 3), T (6 (n-1)^3, 4)."""
    X, T, _ = grid_gel(n, n, n, size=(2 * radius, 2 * radius, 2 * radius))
    P = X - radius
    inf = np.abs(P).max(axis=1)
    two = np.linalg.norm(P, axis=1)
    scale = np.where(two > 0, inf / np.where(two > 0, two, 1.0), 1.0)
    X = P * scale[:, None] + np.asarray(center, dtype=np.float64)
    return X, T


# ----------------------------------------------------------------------------
# Indenter shapes (closed or open triangle meshes in a local frame)
# ----------------------------------------------------------------------------

def icosphere(subdiv: int, radius: float):
    """Icosphere: icosahedron, each subdivision splits a triangle into 4 and
    projects the new vertices onto the sphere. Faces oriented outward."""
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    base = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            base += [(0.0, s1, s2 * phi), (s1, s2 * phi, 0.0), (s2 * phi, 0.0, s1)]
    V = np.array(base, dtype=np.float64)
    # faces = triples of mutually adjacent vertices (edge length 2)
    n = len(V)
    D = np.linalg.norm(V[:, None, :] - V[None, :, :], axis=2)
    adj = np.abs(D - 2.0) < 1e-9
    faces = []
    for i in range(n):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            for k in range(j + 1, n):
                if adj[i, k] and adj[j, k]:
                    a, b, c = V[i], V[j], V[k]
                    if np.dot(np.cross(b - a, c - a), a + b + c) > 0:
                        faces.append((i, j, k))
                    else:
                        faces.append((i, k, j))
    V = V / np.linalg.norm(V, axis=1, keepdims=True)
    F = np.array(faces, dtype=np.int64)
    verts = [tuple(v) for v in V]
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = np.array(verts[a]) + np.array(verts[b])
                m = m / np.linalg.norm(m)
                cache[key] = len(verts)
                verts.append(tuple(m))
            return cache[key]

        nf = []
        for a, b, c in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = np.array(nf, dtype=np.int64)
    V = np.array(verts, dtype=np.float64) * radius
    return V, F.astype(np.int32)


def cylinder(radius: float, length: float, segments: int = 32, rings: int = 24):
    """Capped cylinder with its axis along x, centred at the origin.
    `rings` splits the length so side triangles stay near the gel spacing."""
    V = []
    for r in range(rings + 1):
        x = -0.5 * length + length * r / rings
        for s in range(segments):
            t = 2.0 * math.pi * s / segments
            V.append((x, radius * math.cos(t), radius * math.sin(t)))
    c0 = len(V)
    V.append((-0.5 * length, 0.0, 0.0))
    c1 = len(V)
    V.append((0.5 * length, 0.0, 0.0))
    F = []
    for r in range(rings):
        for s in range(segments):
            a = r * segments + s
            b = r * segments + (s + 1) % segments
            c = (r + 1) * segments + s
            d = (r + 1) * segments + (s + 1) % segments
            F += [(a, b, d), (a, d, c)]
    last = rings * segments
    for s in range(segments):
        F.append((c0, (s + 1) % segments, s))
        F.append((c1, last + s, last + (s + 1) % segments))
    V = np.array(V, dtype=np.float64)
    F = np.array(F, dtype=np.int32)
    return _orient_outward(V, F)


def box(side: float, target_edge: float = 1.25e-3):
    """Closed cube of edge `side` centred at the origin; each face is split into
    k*k quads (k = round(side/target_edge)), two triangles per quad."""
    k = max(1, int(round(side / target_edge)))
    pts = {}
    V = []
    F = []

    def vid(p):
        key = tuple(int(round(c)) for c in p)
        if key not in pts:
            pts[key] = len(V)
            V.append(key)
        return pts[key]

    # lattice coordinates in [0, k]^3
    for axis in range(3):
        for hi in (0, k):
            u, w = [a for a in range(3) if a != axis]
            for i in range(k):
                for j in range(k):
                    quad = []
                    for di, dj in ((0, 0), (1, 0), (1, 1), (0, 1)):
                        p = [0, 0, 0]
                        p[axis] = hi
                        p[u] = i + di
                        p[w] = j + dj
                        quad.append(vid(p))
                    F += [(quad[0], quad[1], quad[2]), (quad[0], quad[2], quad[3])]
    V = (np.array(V, dtype=np.float64) / k - 0.5) * side
    F = np.array(F, dtype=np.int32)
    return _orient_outward(V, F)


def heightfield_plate(rng: np.random.Generator, nxp: int = 128, nyp: int = 128,
                      extent=(0.024, 0.029), gel_size=GEL_SIZE):
    """Open bumpy sheet over the gel plus a 2 mm margin. Gaussian bumps point
    down (toward the gel). Returns V, F in a frame whose x/y origin is the gel
    corner; z = 0 is the flat level, bumps go to negative z."""
    nb = int(rng.integers(3, 13))
    sig = rng.uniform(0.3e-3, 1.0e-3, nb)
    hgt = rng.uniform(0.05e-3, 0.3e-3, nb)
    cx = rng.uniform(0.0, gel_size[0], nb)
    cy = rng.uniform(0.0, gel_size[1], nb)
    x0 = 0.5 * gel_size[0] - 0.5 * extent[0]
    y0 = 0.5 * gel_size[1] - 0.5 * extent[1]
    xs = x0 + extent[0] * np.arange(nxp) / (nxp - 1)
    ys = y0 + extent[1] * np.arange(nyp) / (nyp - 1)
    GX, GY = np.meshgrid(xs, ys, indexing="xy")
    Z = np.zeros_like(GX)
    for b in range(nb):
        Z -= hgt[b] * np.exp(-((GX - cx[b]) ** 2 + (GY - cy[b]) ** 2) / (2.0 * sig[b] ** 2))
    V = np.stack([GX.ravel(), GY.ravel(), Z.ravel()], axis=1)
    F = []
    for j in range(nyp - 1):
        for i in range(nxp - 1):
            a = i + nxp * j
            b = a + 1
            c = a + nxp
            d = c + 1
            # normals point down (-z), toward the gel
            F += [(a, d, b), (a, c, d)]
    return V.astype(np.float64), np.array(F, dtype=np.int32)


def _orient_outward(V, F):
    """Flip faces whose normal points toward the centroid (convex shapes)."""
    cen = V.mean(axis=0)
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    n = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", n, (a + b + c) / 3.0 - cen) < 0
    F = F.copy()
    F[flip, 1], F[flip, 2] = F[flip, 2].copy(), F[flip, 1].copy()
    return V, F


# ----------------------------------------------------------------------------
# Poses
# ----------------------------------------------------------------------------

def rotation(axis, angle: float) -> np.ndarray:
    """Rotation matrix about a unit axis (Rodrigues)."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def pose_matrix(R: np.ndarray, c) -> np.ndarray:
    """Row-major 3x4 rigid transform [R | c]."""
    P = np.zeros((3, 4), dtype=np.float64)
    P[:, :3] = R
    P[:, 3] = c
    return P


def apply_pose(P: np.ndarray, Y: np.ndarray) -> np.ndarray:
    return Y @ P[:, :3].T + P[:, 3]


# ----------------------------------------------------------------------------
# Scene container and the workloads
# ----------------------------------------------------------------------------

@dataclass
class Scene:
    """One gel + indenter problem and its per-step indenter poses."""
    name: str
    X: np.ndarray            # (n,3) gel rest positions
    T: np.ndarray            # (m,4) int32 tets
    fixed: np.ndarray        # (n,) uint8 Dirichlet mask
    Y: np.ndarray            # (k,3) indenter vertices, local frame
    F: np.ndarray            # (f,3) int32 indenter triangles
    poses: np.ndarray        # (steps+1, 3, 4): pose 0 = initial, pose t = target at step t
    dt: float
    E: float = E_YOUNG
    nu: float = NU
    rho: float = RHO
    dhat: float = DHAT
    kappa: float = KAPPA
    k_target: float = K_TARGET
    newton_tol: float = 1e-6
    gravity: tuple = (0.0, 0.0, 0.0)
    self_contact: bool = True
    meta: dict = field(default_factory=dict)
    attached: np.ndarray | None = None    # (n,) uint8: gel vertices held by the sensor case
    case_poses: np.ndarray | None = None  # (steps+1, 3, 4): case pose per step

    @property
    def n_steps(self) -> int:
        return len(self.poses) - 1

    @property
    def bbox_diag(self) -> float:
        """Rest-gel bounding-box diagonal L, used to normalise errors."""
        return float(np.linalg.norm(self.X.max(axis=0) - self.X.min(axis=0)))


def _descent_poses(R, Y, gel_top, center_xy, depth, steps, extra=None, gap=DHAT):
    """Lowest indenter point starts `gap` (dhat) above the gel top and descends
    `depth` in `steps` equal increments; `extra` appends (direction, distance,
    steps) of tangential motion after the descent."""
    Yr = Y @ R.T
    cz = gel_top + gap - Yr[:, 2].min()
    c0 = np.array([center_xy[0], center_xy[1], cz])
    poses = [pose_matrix(R, c0)]
    for t in range(1, steps + 1):
        poses.append(pose_matrix(R, c0 - np.array([0, 0, depth * t / steps])))
    if extra is not None:
        direction, dist, nsteps = extra
        cl = poses[-1][:, 3].copy()
        d = np.asarray(direction, dtype=np.float64)
        for t in range(1, nsteps + 1):
            poses.append(pose_matrix(R, cl + d * dist * t / nsteps))
    return np.stack(poses)


def config1(seed: int = 0) -> Scene:
    """16x20x4 gel, icosphere-2 r=5 mm centred, 1 mm over 10 steps, dt=1e-2."""
    X, T, fixed = grid_gel(16, 20, 4)
    Y, F = icosphere(2, 5e-3)
    poses = _descent_poses(np.eye(3), Y, GEL_SIZE[2], (GEL_SIZE[0] / 2, GEL_SIZE[1] / 2), 1e-3, 10)
    return Scene("c1_16x20x4_icosphere", X, T, fixed, Y, F, poses, dt=1e-2, meta={"seed": seed})


INDENTER_KINDS = ("cylinder", "box_edge", "plate")


def config2(seed: int = 0, grid=(40, 50, 8), steps: int = 50) -> Scene:
    """40x50x8 gel; indenter kind = seed % 3 (cylinder, cube edge, plate);
    1.5 mm over 50 steps, dt=5e-3."""
    rng = np.random.default_rng(seed)
    kind = INDENTER_KINDS[seed % 3]
    X, T, fixed = grid_gel(*grid)
    cxy = (GEL_SIZE[0] / 2, GEL_SIZE[1] / 2)
    if kind == "cylinder":
        r = float(rng.uniform(2e-3, 6e-3))
        Y, F = cylinder(r, 30e-3)
        R = np.eye(3)
        meta = {"radius": r}
    elif kind == "box_edge":
        s = float(rng.uniform(4e-3, 10e-3))
        Y, F = box(s)
        R = rotation((1, 0, 0), math.pi / 4)
        meta = {"side": s}
    else:
        Y, F = heightfield_plate(rng)
        R = np.eye(3)
        cxy = (0.0, 0.0)   # plate coordinates are already in the gel frame
        meta = {}
    poses = _descent_poses(R, Y, GEL_SIZE[2], cxy, 1.5e-3, steps)
    meta.update({"seed": seed, "kind": kind})
    return Scene(f"c2_{grid[0]}x{grid[1]}x{grid[2]}_{kind}_s{seed}", X, T, fixed, Y, F, poses,
                 dt=5e-3, meta=meta)


def config3_scene(i: int, steps: int = 20) -> Scene:
    """Scene i of the 256-scene batch: grid U{12..40}xU{15..50}xU{3..8}, random
    icosphere/cylinder/box with tilt <= 20 deg, depth U[0.5,2] mm over 20 steps."""
    return uneven_scene(1000 + i, steps=steps)


def uneven_scene(seed: int, steps: int = 20, grid=None, prefix: str = "c3") -> Scene:
    """A scene of the uneven batch distribution drawn from `seed`; `grid`
    overrides the drawn resolution (the draws stay the same)."""
    rng = np.random.default_rng(seed)
    nx = int(rng.integers(12, 41))
    ny = int(rng.integers(15, 51))
    nz = int(rng.integers(3, 9))
    if grid is not None:
        nx, ny, nz = grid
    i = seed - 1000
    X, T, fixed = grid_gel(nx, ny, nz)
    kind = ("icosphere", "cylinder", "box")[int(rng.integers(0, 3))]
    if kind == "icosphere":
        Y, F = icosphere(int(rng.integers(2, 4)), float(rng.uniform(3e-3, 8e-3)))
    elif kind == "cylinder":
        Y, F = cylinder(float(rng.uniform(2e-3, 6e-3)), 30e-3)
    else:
        Y, F = box(float(rng.uniform(4e-3, 10e-3)))
    axis = rng.normal(size=3)
    R = rotation(axis, math.radians(float(rng.uniform(0.0, 20.0))))
    depth = float(rng.uniform(0.5e-3, 2e-3))
    poses = _descent_poses(R, Y, GEL_SIZE[2], (GEL_SIZE[0] / 2, GEL_SIZE[1] / 2), depth, steps)
    return Scene(f"{prefix}_{i}_{nx}x{ny}x{nz}_{kind}", X, T, fixed, Y, F, poses, dt=1e-2,
                 meta={"i": i, "seed": seed, "kind": kind, "depth": depth})


def serving_scene(env: int, large: bool, steps: int = 20) -> Scene:
    """Environment `env` of the serving workload: the uneven batch
    distribution from seed 5000 + env, at 80x100x16 for the large ones."""
    return uneven_scene(5000 + env, steps=steps, grid=(80, 100, 16) if large else None, prefix="c4")


def config5(indent_steps: int = 40, slide_steps: int = 160) -> Scene:
    """80x100x16 gel, icosphere-4 r=8 mm: 1 mm indent then 5 mm slide in +x."""
    X, T, fixed = grid_gel(80, 100, 16)
    Y, F = icosphere(4, 8e-3)
    poses = _descent_poses(np.eye(3), Y, GEL_SIZE[2], (GEL_SIZE[0] / 2 - 2.5e-3, GEL_SIZE[1] / 2),
                           1e-3, indent_steps, extra=((1, 0, 0), 5e-3, slide_steps))
    return Scene("c5_80x100x16_icosphere4", X, T, fixed, Y, F, poses, dt=1e-2,
                 meta={"mu": 0.5, "eps_v": 1e-3, "radius": 8e-3})


# Soft-ball workloads at the mesh sizes of the paper's GIPC timing table
# (Table 3: 1029/3717, 7900/40370, 12509/66563 vertices/tets), counted here
# as gel + ball: (gel grid, ball grid points per axis).
SOFT_BALL_SIZES = {
    "tiny": ((6, 6, 3), 5),        # 233 v, 918 t (parity tests)
    "small": ((12, 13, 3), 8),     # 980 v, 3642 t
    "medium": ((28, 28, 4), 17),   # 8049 v, 37698 t
    "large": ((30, 30, 5), 20),    # 12500 v, 61338 t
}


def soft_ball_scene(size: str = "small", radius: float = 5e-3, depth: float = 2.0e-3, steps: int = 20,
                    slide: float = 0.0, slide_steps: int = 0, mu: float = 0.0, dt: float = 1e-2) -> Scene:
    """Two deformable bodies in contact: the gel pad (bottom fixed) and a soft
    ball resting dhat/2 above its centre (inside the barrier's range, so the
    gel holds it from the first step), squeezed by a rigid plate (a box
    indenter dhat/2 above the ball) that descends `depth` over `steps`; with
    `slide` > 0 the plate then moves along +x over `slide_steps` (with
    friction mu the ball rolls on the gel). Gel-ball contact is self-contact
    of the deformable set."""
    (gx, gy, gz), nb = SOFT_BALL_SIZES[size]
    Xg, Tg, fixed = grid_gel(gx, gy, gz)
    top = GEL_SIZE[2]
    c = np.array([GEL_SIZE[0] / 2, GEL_SIZE[1] / 2, top + radius])
    Xb, Tb = soft_ball(nb, radius, c)
    Xb[:, 2] += top + 0.5 * DHAT - Xb[:, 2].min()
    X = np.concatenate([Xg, Xb])
    T = np.concatenate([Tg, Tb + len(Xg)]).astype(np.int32)
    fixed = np.concatenate([fixed, np.zeros(len(Xb), dtype=np.uint8)])
    Y, F = box(4 * radius, target_edge=radius / 2)
    ball_top = Xb[:, 2].max()
    R = np.eye(3)
    extra = ((1, 0, 0), slide, slide_steps) if slide > 0 else None
    poses = _descent_poses(R, Y, ball_top - 0.5 * DHAT, (c[0], c[1]), depth, steps, extra=extra)
    meta = {"kind": "soft_ball", "size": size, "n_gel": len(Xg), "n_ball": len(Xb)}
    if mu > 0:
        meta.update({"mu": mu, "eps_v": 1e-3})
    return Scene(f"soft_ball_{size}", X, T, fixed, Y, F, poses, dt=dt, meta=meta)


def attached_scene(grid=(16, 20, 4), depth: float = 1.0e-3, steps: int = 10, tilt_deg: float = 0.0,
                   radius: float = 5e-3, dt: float = 1e-2) -> Scene:
    """The sensor moves, the object stays: the gel's bottom layer is held by
    the sensor case (attached, not fixed) and the case lifts the gel by
    `depth` over `steps` (tilting by `tilt_deg` about the x axis through the
    bottom centre along the way) into a static icosphere whose lowest point
    starts dhat above the gel top. The indenter keeps its initial pose."""
    X, T, bottom = grid_gel(*grid)
    fixed = np.zeros(len(X), dtype=np.uint8)
    Y, F = icosphere(2, radius)
    R = np.eye(3)
    # the sphere hangs above the gel centre with its lowest point dhat above the top
    c = np.array([GEL_SIZE[0] / 2, GEL_SIZE[1] / 2, GEL_SIZE[2] + DHAT - Y[:, 2].min()])
    P0 = pose_matrix(R, c)
    poses = np.stack([P0] * (steps + 1))
    # the case: the gel moves up towards the sphere (the sensor pressed onto it)
    cases = []
    for t in range(steps + 1):
        a = math.radians(tilt_deg) * t / steps
        Rc = rotation((1, 0, 0), a)
        ctr = np.array([GEL_SIZE[0] / 2, GEL_SIZE[1] / 2, 0.0])
        # rotate about the bottom centre, then lift
        off = ctr - Rc @ ctr + np.array([0, 0, depth * t / steps])
        cases.append(pose_matrix(Rc, off))
    return Scene(f"attached_{grid[0]}x{grid[1]}x{grid[2]}", X, T, fixed, Y, F, poses, dt=dt,
                 attached=bottom.copy(), case_poses=np.stack(cases), meta={"kind": "attached"})


def tiny_scene(grid=(4, 4, 3), radius=2e-3, subdiv=1, depth=0.3e-3, steps=3, dt=1e-2,
               self_contact=True) -> Scene:
    """A very small gel and icosphere for brute-force checks."""
    size = (0.004, 0.004, 0.002)
    X, T, fixed = grid_gel(*grid, size=size)
    Y, F = icosphere(subdiv, radius)
    poses = _descent_poses(np.eye(3), Y, size[2], (size[0] / 2, size[1] / 2), depth, steps)
    return Scene(f"tiny_{grid[0]}x{grid[1]}x{grid[2]}", X, T, fixed, Y, F, poses, dt=dt,
                 self_contact=self_contact)


def tiny_slide_scene(mu: float = 0.5, eps_v: float = 1e-3, grid=(6, 5, 4), press_steps=3, slide_steps=4,
                     slide=0.4e-3) -> Scene:
    """A small gel pressed 0.3 mm by an icosphere that then slides along +x
    (lagged friction with coefficient mu, velocity threshold eps_v)."""
    size = (0.004, 0.004, 0.002)
    X, T, fixed = grid_gel(*grid, size=size)
    Y, F = icosphere(2, 1.5e-3)
    poses = _descent_poses(np.eye(3), Y, size[2], (size[0] / 2 - 0.2e-3, size[1] / 2), 0.3e-3, press_steps,
                           extra=((1, 0, 0), slide, slide_steps))
    return Scene(f"tiny_slide_mu{mu}", X, T, fixed, Y, F, poses, dt=1e-2, meta={"mu": mu, "eps_v": eps_v})



# Hertz check: a rigid sphere pressed quasi-statically into a thick block
# (half-space Hertz contact needs the contact radius a = sqrt(R delta) well
# below the block's thickness and width). The barrier range is cut to 10 um
# in this scene so the contact gap stays far below the smallest depth.
HERTZ_SIZE = (0.030, 0.030, 0.015)
HERTZ_DHAT = 1e-5


def hertz_scene(grid=(41, 41, 21), subdiv: int = 5, radius: float = 0.02, depth: float = 0.5e-3,
                steps: int = 10, dt: float = 1.0, newton_tol: float = 1e-8, size=HERTZ_SIZE) -> Scene:
    """Block `size` (bottom fixed) meshed as a Kuhn grid, icosphere of `radius`
    starting dhat above the top centre and descending `depth` over `steps`
    equal increments; quasi-static (dt = 1 s, no gravity), no friction, no
    self-contact, dhat = 10 um, kappa = 1e4, Newton tolerance `newton_tol`."""
    X, T, fixed = grid_gel(*grid, size=size)
    Y, F = icosphere(subdiv, radius)
    poses = _descent_poses(np.eye(3), Y, size[2], (size[0] / 2, size[1] / 2), depth, steps, gap=HERTZ_DHAT)
    return Scene(f"hertz_{grid[0]}x{grid[1]}x{grid[2]}_R{radius * 1e3:g}mm", X, T, fixed, Y, F, poses, dt=dt,
                 dhat=HERTZ_DHAT, newton_tol=newton_tol, self_contact=False,
                 meta={"kind": "hertz", "radius": radius, "top": size[2], "center": (size[0] / 2, size[1] / 2),
                       "gap0": HERTZ_DHAT})


def pressed_state(sc: Scene, step: int, gap_frac: float = 0.5):
    """A constructed contact state for one-iterate checks: the indenter at its
    pose of `step` (rigid, no lag), a spherical indenter (meta 'radius',
    centred on the pose's translation) and the gel's top surface pushed under
    it to `gap_frac` dhat below the sphere where the undeformed top would
    reach into it (contact radius a), falling off as (a / r)^4 outside; the
    vertical displacement decays linearly to zero at the fixed bottom, and
    velocities are zero. Only +, -, *, / and sqrt are used, so the state is
    the same bits on every machine. Returns (x (n_all, 3), v (n_all, 3))."""
    R = float(sc.meta["radius"])
    P = sc.poses[step]
    c = P[:, 3]
    X = sc.X
    top = float(X[:, 2].max())
    bottom = float(X[:, 2].min())
    r2 = (X[:, 0] - c[0]) ** 2 + (X[:, 1] - c[1]) ** 2
    inside = r2 < R * R
    zs = np.where(inside, c[2] - np.sqrt(np.where(inside, R * R - r2, 0.0)), np.inf)
    pen = top - zs                      # > 0 where the undeformed top reaches into the sphere
    g = gap_frac * sc.dhat
    a2 = float(r2[pen >= 0].max()) if np.any(pen >= 0) else 0.0
    w = np.where(pen >= 0, -(pen + g), 0.0)
    if a2 > 0:
        q = a2 / np.maximum(r2, a2)
        w = np.where(pen >= 0, w, -g * q * q)
    x = X.copy()
    x[:, 2] += w * (X[:, 2] - bottom) / (top - bottom)
    y = apply_pose(P, sc.Y)
    xa = np.concatenate([x, y])
    return xa, np.zeros_like(xa)
