"""Seeded synthetic inputs for the refined KBC workloads.

This module holds geometry and initial fields only -- no part of the method's
arithmetic (no equilibrium, collision, coupling or lattice table).  Both the HIP
library and the CPU oracle are driven from the same generated inputs.

Workloads (stand-ins for the paper's channel, sphere and block-refined cases,
Sec. IV.A; the paper's datasets are not used):

  tgv2d      D2Q9 periodic Taylor-Green vortex, one centred refined patch.
  channel3d  D3Q27 channel, periodic x/z, walls in y, refined near-wall slabs,
             constant body force, seeded velocity perturbations.
  sphere3d   D3Q27 flow past a sphere, three nested levels, inlet/outflow.
  forest3d   D3Q27 periodic block forest of 16^3-cell blocks over four levels
             with 2:1 balance and seeded per-node velocities in the ball |u|<=0.05.
  cylinder2d D2Q9 channel with a cylinder inside a refined patch.

Conventions: level-l coordinates are integers in level-l spacing; a dense field of
a level covers that level's index box (lo, n) with numpy shape (n_z, n_y, n_x) in
3-D or (n_y, n_x) in 2-D; vector fields carry a leading component axis.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Tuple

import numpy as np

SEED = 1608

FACE_WALL, FACE_INLET, FACE_OUTFLOW = 1, 2, 3


def rng(seed: int = SEED) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Spec:
    name: str
    D: int
    N: Tuple[int, ...]
    periodic: Tuple[bool, ...]
    nu0: float
    levels: int
    boxes: Dict[int, List[Tuple[Tuple[int, ...], Tuple[int, ...]]]] = field(default_factory=dict)
    faces: Dict[int, Tuple[int, Tuple[float, float, float]]] = field(default_factory=dict)
    # level -> (centre in level coords, radius in level units, kind "sphere"/"disc")
    bodies: Dict[int, Tuple[Tuple[float, ...], float]] = field(default_factory=dict)
    force: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    init: Optional[Callable] = None  # (level, lo, n) -> (rho, u, noise or None)
    U: float = 0.05  # reference velocity
    body_level: Optional[int] = None
    body_diameter: Optional[float] = None  # in body-level units

    @property
    def Q(self):
        return 9 if self.D == 2 else 27


def coords(lo, n, D):
    """Integer level coordinates of a dense box, each of numpy shape."""
    axes = [np.arange(lo[a], lo[a] + n[a]) for a in range(D)]
    grids = np.meshgrid(*axes[::-1], indexing="ij")  # z/y, ..., x order
    return grids[::-1]  # x, y, (z)


def body_mask(spec: Spec, level: int, lo, n):
    """uint8 solid mask of the spec's body over a dense level box."""
    if level not in spec.bodies:
        return None
    centre, radius = spec.bodies[level]
    X = coords(lo, n, spec.D)
    r2 = sum((X[a].astype(np.float64) - centre[a]) ** 2 for a in range(spec.D))
    return (r2 <= radius * radius).astype(np.uint8)


def solid_box(spec: Spec, level: int):
    """(lo, mask) covering the body with one node of margin, or None."""
    if level not in spec.bodies:
        return None
    centre, radius = spec.bodies[level]
    lo = [int(math.floor(centre[a] - radius)) - 1 for a in range(spec.D)]
    hi = [int(math.ceil(centre[a] + radius)) + 1 for a in range(spec.D)]
    n = [hi[a] - lo[a] + 1 for a in range(spec.D)]
    return lo, body_mask(spec, level, lo, n)


def apply(spec: Spec, lat) -> None:
    """Describe the workload to a lattice object (HIP library or oracle binding):
    faces, refinement boxes, solids and uniform force, then finalize."""
    for face, (kind, u) in spec.faces.items():
        lat.set_face(face, kind, u)
    for level in sorted(spec.boxes):
        for lo, hi in spec.boxes[level]:
            lat.add_box(level, lo, hi)
    for level in spec.bodies:
        lo, mask = solid_box(spec, level)
        lat.set_solid(level, lo, mask)
    lat.set_force_uniform(spec.force)
    lat.finalize()


def fields(spec: Spec, level: int, lo, n):
    """Initial (rho, u, noise) for a level's dense index box."""
    return spec.init(level, lo, n)


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------

def tgv2d(n0: int = 64, patch=(16, 48), u0: float = 0.05, nu0: float = 0.01, noise: float = 0.0,
          seed: int = SEED) -> Spec:
    """Periodic n0 x n0 Taylor-Green vortex, refined patch [patch]^2 (coarse units)."""
    k = 2.0 * math.pi / n0

    def init(level, lo, n):
        s = 2.0 ** level
        X, Y = coords(lo, n, 2)
        x, y = X / s, Y / s
        ux = -u0 * np.cos(k * x) * np.sin(k * y)
        uy = u0 * np.sin(k * x) * np.cos(k * y)
        rho = 1.0 - 0.75 * u0 * u0 * (np.cos(2 * k * x) + np.cos(2 * k * y))
        nz = None
        if noise:
            nz = noise * rng(seed + 100 * level).uniform(-1.0, 1.0, size=(9,) + rho.shape)
        return rho, np.stack([ux, uy]), nz

    boxes = {1: [((2 * patch[0], 2 * patch[0]), (2 * patch[1], 2 * patch[1]))]} if patch else {}
    return Spec("tgv2d", 2, (n0, n0), (True, True), nu0, 2 if patch else 1, boxes, init=init, U=u0)


def channel3d(nx: int = 128, ny: int = 64, nz: int = 64, slab: int = 8, nu0: float = 6.0e-4, ub: float = 0.05,
              re_tau: float = 180.0, pert: float = 0.05, seed: int = SEED, levels: int = 2) -> Spec:
    """Channel: periodic x, z; walls at y = -1/4 and ny-3/4 (coarse) resolved on the
    fine slabs; fine slabs y in [0, slab] and [ny-1-slab, ny-1] (coarse)."""
    # half width in coarse units: fine nodes 0..2(ny-1), walls half a fine spacing outside
    delta = (2 * (ny - 1) + 1) / 4.0
    g = re_tau ** 2 * nu0 ** 2 / delta ** 3

    def init(level, lo, n):
        shp = tuple(int(v) for v in n[:3][::-1])
        r = rng(seed + 7919 * level)
        xi = r.uniform(-1.0, 1.0, size=(3,) + shp)
        u = pert * ub * xi
        u[0] += ub
        return np.ones(shp), u, None

    Xf = 2 * nx - 1
    Zf = 2 * nz - 1
    boxes = {1: [((0, 0, 0), (Xf, 2 * slab, Zf)), ((0, 2 * (ny - 1 - slab), 0), (Xf, 2 * (ny - 1), Zf))]}
    if levels == 1:
        boxes = {}
    sp = Spec("channel3d", 3, (nx, ny, nz), (True, False, True), nu0, levels, boxes,
              faces={2: (FACE_WALL, (0, 0, 0)), 3: (FACE_WALL, (0, 0, 0))}, force=(g, 0.0, 0.0), init=init, U=ub)
    return sp


def sphere3d(nx: int = 256, ny: int = 128, nz: int = 128, U: float = 0.05, Re: float = 300.0, D_fine: float = 20.0,
             l1=((48, 48, 48), (112, 80, 80)), l2=((56, 56, 56), (88, 72, 72)), centre=(64, 64, 64),
             noise: float = 0.0, seed: int = SEED) -> Spec:
    """Sphere of diameter D_fine (finest-level units) at `centre` (coarse coords);
    three levels with boxes l1, l2 in coarse coordinates; inlet at x=0, outflow at
    x=nx-1, periodic in y and z."""
    nu2 = U * D_fine / Re
    nu0 = nu2 / 4.0

    def init(level, lo, n):
        shp = tuple(int(v) for v in n[:3][::-1])
        u = np.zeros((3,) + shp)
        u[0] = U
        nzs = noise * rng(seed + 13 * level).uniform(-1.0, 1.0, size=(27,) + shp) if noise else None
        return np.ones(shp), u, nzs

    def sc(b, s):
        return tuple(int(v) * s for v in b)

    boxes = {1: [(sc(l1[0], 2), sc(l1[1], 2))], 2: [(sc(l2[0], 4), sc(l2[1], 4))]}
    sp = Spec("sphere3d", 3, (nx, ny, nz), (False, True, True), nu0, 3, boxes,
              faces={0: (FACE_INLET, (U, 0.0, 0.0)), 1: (FACE_OUTFLOW, (0.0, 0.0, 0.0))},
              bodies={2: (tuple(4.0 * c for c in centre), D_fine / 2.0)}, init=init, U=U, body_level=2,
              body_diameter=D_fine)
    return sp


def sphere_paper3d(U: float = 0.05, Re: float = 3700.0, D_fine: float = 120.0) -> Spec:
    """The sphere at the paper's own scale (Sec. IV, sphere at Re = 3700): four levels,
    diameter D = 120 finest units, domain about 30D x 20D x 20D (448 x 296 x 296 coarse: the
    largest that keeps one level's population buffer under the 4 GiB that 32-bit brick
    offsets address), three nested boxes around the sphere and its near wake (coarse
    coordinates below), about 96e6 nodes in all.  Inlet at x = 0, outflow at x = nx - 1,
    periodic in y and z; uniform initial velocity U.  The box extents are this
    workload's own (the paper does not list them)."""
    nx, ny, nz = 448, 296, 296
    centre = (150.0, 148.0, 148.0)
    nu3 = U * D_fine / Re
    nu0 = nu3 / 8.0
    coarse_boxes = {1: ((104, 108, 108), (264, 188, 188)), 2: ((120, 122, 122), (220, 174, 174)),
                    3: ((130, 132, 132), (190, 164, 164))}

    def init(level, lo, n):
        shp = tuple(int(v) for v in n[:3][::-1])
        u = np.zeros((3,) + shp)
        u[0] = U
        return np.ones(shp), u, None

    boxes = {l: [(tuple(v << l for v in b[0]), tuple(v << l for v in b[1]))] for l, b in coarse_boxes.items()}
    return Spec("sphere_paper3d", 3, (nx, ny, nz), (False, True, True), nu0, 4, boxes,
                faces={0: (FACE_INLET, (U, 0.0, 0.0)), 1: (FACE_OUTFLOW, (0.0, 0.0, 0.0))},
                bodies={3: (tuple(8.0 * c for c in centre), D_fine / 2.0)}, init=init, U=U, body_level=3,
                body_diameter=D_fine)


def _forest(root: Tuple[int, int, int], counts: Tuple[int, ...], r: np.random.Generator):
    """Nested compact clusters of refined blocks.  Level l blocks have 16 level-l cells
    per axis; refining a block produces its 8 children.  A block is refined only if all
    26 neighbours at its level exist, which enforces 2:1 balance across faces, edges and
    corners (periodic).  Returns the refined block index sets per level."""
    dims = [np.array(root, dtype=np.int64)]
    refined = []
    present = {tuple(b) for b in np.ndindex(*root)}
    for lvl, cnt in enumerate(counts):
        dim = dims[lvl]
        cand = []
        for b in present:
            ok = True
            for off in np.ndindex(3, 3, 3):
                nb = tuple((b[a] + off[a] - 1) % dim[a] for a in range(3))
                if nb not in present:
                    ok = False
                    break
            if ok:
                cand.append(b)
        if len(cand) < cnt:
            raise ValueError("forest: not enough balanced candidates at level %d" % lvl)
        cand.sort()

        def pdist(b, centre):
            d = np.abs(np.array(b, dtype=np.float64) - centre)
            d = np.minimum(d, dim - d)
            return float(np.sum(d * d))

        # cluster around a block corner so that the chosen blocks are compact and the
        # next level has balanced candidates; retry with other corners if needed
        chosen = None
        for _attempt in range(64):
            centre = np.array(cand[int(r.integers(len(cand)))], dtype=np.float64) + 0.5
            jitter = r.uniform(0, 0.5, size=len(cand))
            order = sorted(range(len(cand)), key=lambda i: pdist(cand[i], centre) + jitter[i])
            chosen = [cand[i] for i in order[:cnt]]
            if lvl + 1 >= len(counts) or _balanced_children(chosen, dim * 2) >= counts[lvl + 1]:
                break
        refined.append(sorted(chosen))
        children = set()
        for b in chosen:
            for off in np.ndindex(2, 2, 2):
                children.add(tuple(2 * b[a] + off[a] for a in range(3)))
        present = children
        dims.append(dim * 2)
    return refined


def _balanced_children(chosen, dim):
    children = set()
    for b in chosen:
        for off in np.ndindex(2, 2, 2):
            children.add(tuple(2 * b[a] + off[a] for a in range(3)))
    n = 0
    for b in children:
        if all(tuple((b[a] + off[a] - 1) % dim[a] for a in range(3)) in children for off in np.ndindex(3, 3, 3)):
            n += 1
    return n


def forest3d(root=(9, 5, 5), counts=(21, 14, 6), umax: float = 0.05, nu0: float = 1.0e-3, seed: int = SEED,
             block: int = 16) -> Spec:
    """Periodic block forest: root blocks of `block` coarse cells; `counts` blocks are
    refined at levels 0, 1, 2.  With the defaults the leaves per level are
    (204, 154, 106, 48) = 512 blocks of 16^3 cells."""
    r = rng(seed)
    refined = _forest(tuple(root), tuple(counts), r)
    L = len(counts) + 1
    boxes = {}
    for lvl, blocks in enumerate(refined):
        # a refined level-lvl block b covers level-(lvl+1) nodes [2*block*b, 2*block*(b+1)]
        bl = []
        for b in blocks:
            lo = tuple(2 * block * int(v) for v in b)
            hi = tuple(2 * block * (int(v) + 1) for v in b)
            bl.append((lo, hi))
        boxes[lvl + 1] = bl
    N = tuple(block * int(v) for v in root)

    def init(level, lo, n):
        shp = tuple(int(v) for v in n[:3][::-1])
        rr = rng(seed + 104729 * (level + 1))
        tot = int(np.prod(shp))
        out = np.empty((tot, 3))
        filled = 0
        while filled < tot:
            cand = rr.uniform(-umax, umax, size=(2 * (tot - filled) + 16, 3))
            cand = cand[np.sum(cand * cand, axis=1) <= umax * umax]
            take = min(len(cand), tot - filled)
            out[filled:filled + take] = cand[:take]
            filled += take
        u = out.T.reshape((3,) + shp)
        return np.ones(shp), u, None

    sp = Spec("forest3d", 3, N, (True, True, True), nu0, L, boxes, init=init, U=umax)
    sp.leaves = _leaf_counts(root, refined)
    return sp


def _leaf_counts(root, refined):
    n = [int(np.prod(root))]
    for lvl, blocks in enumerate(refined):
        n[lvl] -= len(blocks)
        n.append(8 * len(blocks))
    return tuple(n)


def cylinder2d(nx: int = 256, ny: int = 128, patch=((40, 32), (120, 96)), centre=(64, 64), D_fine: float = 32.0,
               U: float = 0.05, Re: float = 100.0, noise: float = 1.0e-3, seed: int = SEED) -> Spec:
    """Body-force driven channel with walls at y=-1/2 and ny-1/2 (coarse), periodic x,
    cylinder of diameter D_fine (fine units) in a refined patch."""
    nu1 = U * D_fine / Re
    nu0 = nu1 / 2.0
    Fx = 12.0 * nu0 * U / float(ny) ** 2

    def init(level, lo, n):
        shp = tuple(int(v) for v in n[:2][::-1])
        nz = noise * rng(seed + 31 * level).uniform(-1.0, 1.0, size=(9,) + shp) if noise else None
        return np.ones(shp), np.zeros((2,) + shp), nz

    boxes = {1: [((2 * patch[0][0], 2 * patch[0][1]), (2 * patch[1][0], 2 * patch[1][1]))]}
    return Spec("cylinder2d", 2, (nx, ny), (True, False), nu0, 2, boxes,
                faces={2: (FACE_WALL, (0, 0, 0)), 3: (FACE_WALL, (0, 0, 0))},
                bodies={1: ((2.0 * centre[0], 2.0 * centre[1]), D_fine / 2.0)}, force=(Fx, 0.0, 0.0), init=init,
                U=U, body_level=1, body_diameter=D_fine)


def pop_noise(Q: int, shape, amp: float, seed: int) -> np.ndarray:
    """Relative per-population perturbation in [-amp, amp]."""
    return amp * rng(seed).uniform(-1.0, 1.0, size=(Q,) + tuple(shape))


def random_states(D: int, count: int, seed: int, spread: float = 0.5):
    """Generic positive population vectors (raw input for single-node tests):
    independent uniform values in [1-spread, 1+spread] / Q, scaled by a random
    density in [0.8, 1.2].  Far from any equilibrium on purpose."""
    r = rng(seed)
    Q = 9 if D == 2 else 27
    base = r.uniform(1.0 - spread, 1.0 + spread, size=(count, Q)) / Q
    return base * r.uniform(0.8, 1.2, size=(count, 1))
