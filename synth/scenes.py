"""Seeded synthetic inputs shaped like the paper's sensed scenes.

This module only draws random numbers and places them in arrays. It holds none
of the method's arithmetic (no tree, no filter, no distance test), so both the
oracle and the GPU path can take their inputs from it.

The paper's own workloads (MotionBenchMaker scenes, RealSense frames) are not
available; these clouds follow the recipe the paper gives for its throughput
experiment (Sec. VI-A): uniform random sampling of obstacle surfaces, then the
Morton filter.  Every generator computes in float64 and rounds to float32 once.
Seeds are fixed per workload: cloud = 1000*k + 1, queries = 1000*k + 2,
template = 1000*k + 3 for workload k; the batched workload uses 3100 + c for
cloud c and 3200 + c for its queries.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Workspace of the tabletop scenes: x, y in [-1, 1] m, z in [0, 1.5] m.
WORKSPACE = np.array([[-1.0, 1.0], [-1.0, 1.0], [0.0, 1.5]])
# Room scene: 6 m x 6 m x 3 m.
ROOM = np.array([[0.0, 6.0], [0.0, 6.0], [0.0, 3.0]])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_cube_cloud(n: int, seed: int) -> np.ndarray:
    """n points iid uniform in [0, 1]^3, float32 [n, 3]."""
    return _rng(seed).random((n, 3)).astype(np.float32)


def uniform_spheres(m: int, box, r_lo: float, r_hi: float, seed: int,
                    chunk: int = 1 << 22) -> np.ndarray:
    """m spheres (x, y, z, r): centres uniform in `box` ([3, 2] bounds), radii
    uniform in [r_lo, r_hi]; float32 [m, 4].  Drawn in chunks so that 10^8
    spheres fit in host memory."""
    box = np.asarray(box, dtype=np.float64)
    g = _rng(seed)
    out = np.empty((m, 4), dtype=np.float32)
    for s in range(0, m, chunk):
        e = min(m, s + chunk)
        u = g.random((e - s, 4))
        c = box[:, 0] + u[:, :3] * (box[:, 1] - box[:, 0])
        r = r_lo + u[:, 3] * (r_hi - r_lo)
        out[s:e, :3] = c
        out[s:e, 3] = r
    return out


# ----------------------------------------------------------------------------
# Surface primitives
# ----------------------------------------------------------------------------
@dataclass
class Box:
    lo: np.ndarray  # [3]
    size: np.ndarray  # [3]

    def area(self) -> float:
        sx, sy, sz = self.size
        return 2.0 * (sx * sy + sy * sz + sx * sz)

    def sample(self, g: np.random.Generator, k: int) -> np.ndarray:
        sx, sy, sz = self.size
        faces = np.array([sy * sz, sy * sz, sx * sz, sx * sz, sx * sy, sx * sy])
        f = g.choice(6, size=k, p=faces / faces.sum())
        u = g.random((k, 3))
        p = self.lo + u * self.size
        axis = f // 2
        side = f % 2
        p[np.arange(k), axis] = self.lo[axis] + side * self.size[axis]
        return p


@dataclass
class Cylinder:
    cx: float
    cy: float
    z0: float
    radius: float
    height: float

    def area(self) -> float:
        return 2.0 * math.pi * self.radius * self.height + 2.0 * math.pi * self.radius ** 2

    def sample(self, g: np.random.Generator, k: int) -> np.ndarray:
        lat = 2.0 * math.pi * self.radius * self.height
        cap = math.pi * self.radius ** 2
        part = g.choice(3, size=k, p=np.array([lat, cap, cap]) / (lat + 2 * cap))
        th = g.random(k) * 2.0 * math.pi
        rr = np.where(part == 0, self.radius, self.radius * np.sqrt(g.random(k)))
        z = np.where(part == 0, self.z0 + g.random(k) * self.height,
                     np.where(part == 1, self.z0, self.z0 + self.height))
        return np.stack([self.cx + rr * np.cos(th), self.cy + rr * np.sin(th), z], axis=1)


@dataclass
class Plane:
    """Axis-aligned rectangle: fixed coordinate `value` on `axis`, spanning
    `span` ([3, 2]) on the two other axes."""
    axis: int
    value: float
    span: np.ndarray

    def area(self) -> float:
        ext = self.span[:, 1] - self.span[:, 0]
        ext = np.delete(ext, self.axis)
        return float(ext[0] * ext[1])

    def sample(self, g: np.random.Generator, k: int) -> np.ndarray:
        u = g.random((k, 3))
        p = self.span[:, 0] + u * (self.span[:, 1] - self.span[:, 0])
        p[:, self.axis] = self.value
        return p


def _random_boxes(g, count, space, size_lo, size_hi):
    out = []
    for _ in range(count):
        size = g.uniform(size_lo, size_hi, 3)
        lo = space[:, 0] + g.random(3) * (space[:, 1] - space[:, 0] - size)
        out.append(Box(lo, size))
    return out


def _random_cylinders(g, count, space, size_lo, size_hi):
    out = []
    for _ in range(count):
        d = g.uniform(size_lo, size_hi)
        h = g.uniform(size_lo, size_hi)
        rad = d / 2.0
        cx = g.uniform(space[0, 0] + rad, space[0, 1] - rad)
        cy = g.uniform(space[1, 0] + rad, space[1, 1] - rad)
        z0 = g.uniform(space[2, 0], space[2, 1] - h)
        out.append(Cylinder(cx, cy, z0, rad, h))
    return out


def _sample_surfaces(g, prims, n):
    areas = np.array([p.area() for p in prims])
    counts = g.multinomial(n, areas / areas.sum())
    parts = [p.sample(g, int(k)) for p, k in zip(prims, counts) if k > 0]
    pts = np.concatenate(parts, axis=0)
    return pts[g.permutation(len(pts))]


def tabletop_cloud(n: int, seed: int, n_boxes: int = 24, n_cyl: int = 8,
                   size=(0.05, 0.6), noise: float = 0.002) -> np.ndarray:
    """n points on the surfaces of `n_boxes` axis-aligned boxes and `n_cyl`
    vertical cylinders (all sides, diameters and heights uniform in `size`)
    placed fully inside the 2 x 2 x 1.5 m workspace.  Points are split over the
    primitives in proportion to surface area (cylinder caps included), drawn
    uniformly on each surface, then perturbed by iid N(0, noise^2) per axis.
    float32 [n, 3]."""
    g = _rng(seed)
    prims = (_random_boxes(g, n_boxes, WORKSPACE, *size)
             + _random_cylinders(g, n_cyl, WORKSPACE, *size))
    pts = _sample_surfaces(g, prims, n)
    pts = pts + g.normal(0.0, noise, pts.shape)
    return pts.astype(np.float32)


def depth_frame(seed: int = 7001, width: int = 640, height: int = 480, hfov_deg: float = 87.0,
                vfov_deg: float = 58.0, scene_seed: int = 2001) -> np.ndarray:
    """One synthetic depth-camera frame of the tabletop scene (the boxes and
    cylinders of `tabletop_cloud(.., scene_seed)`) inside a 6 x 6 x 3 m room:
    one point per pixel (width x height), where the pixel's ray first meets a
    surface, with depth noise N(0, (0.001 m * depth^2)) along the ray.  The
    camera stands at a seeded point 1.8-2.4 m from the workspace centre at
    1.0-1.6 m height and looks at it, with the field of view of a common
    stereo depth camera (87 x 58 degrees).  float32 [width * height, 3]."""
    gs = _rng(scene_seed)
    boxes = _random_boxes(gs, 24, WORKSPACE, 0.05, 0.6)
    cyls = _random_cylinders(gs, 8, WORKSPACE, 0.05, 0.6)
    g = _rng(seed)
    ang = g.uniform(0.0, 2.0 * math.pi)
    dist = g.uniform(1.8, 2.4)
    cam = np.array([dist * math.cos(ang), dist * math.sin(ang), g.uniform(1.0, 1.6)])
    look = np.array([0.0, 0.0, 0.5]) - cam
    fwd = look / np.linalg.norm(look)
    right = np.cross(fwd, np.array([0.0, 0.0, 1.0]))
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    u = (np.arange(width) + 0.5) / width * 2.0 - 1.0
    v = 1.0 - (np.arange(height) + 0.5) / height * 2.0
    uu, vv = np.meshgrid(u * math.tan(math.radians(hfov_deg) / 2), v * math.tan(math.radians(vfov_deg) / 2))
    d = fwd[None, :] + uu.reshape(-1, 1) * right[None, :] + vv.reshape(-1, 1) * up[None, :]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = cam
    best = np.full(len(d), np.inf)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        for b in boxes:
            t1 = (b.lo - o) * inv
            t2 = (b.lo + b.size - o) * inv
            tn = np.nanmax(np.minimum(t1, t2), axis=1)
            tf = np.nanmin(np.maximum(t1, t2), axis=1)
            hit = (tf >= np.maximum(tn, 0.0)) & (tn > 0.0)
            best = np.where(hit & (tn < best), tn, best)
        for c in cyls:
            ox, oy = o[0] - c.cx, o[1] - c.cy
            a = d[:, 0] ** 2 + d[:, 1] ** 2
            bq = 2.0 * (ox * d[:, 0] + oy * d[:, 1])
            cq = ox * ox + oy * oy - c.radius ** 2
            disc = bq * bq - 4.0 * a * cq
            t = (-bq - np.sqrt(np.maximum(disc, 0.0))) / (2.0 * a)
            z = o[2] + t * d[:, 2]
            hit = (disc >= 0.0) & (t > 0.0) & (z >= c.z0) & (z <= c.z0 + c.height)
            best = np.where(hit & (t < best), t, best)
            for zc in (c.z0, c.z0 + c.height):
                t = (zc - o[2]) * inv[:, 2]
                x = o[0] + t * d[:, 0] - c.cx
                y = o[1] + t * d[:, 1] - c.cy
                hit = (t > 0.0) & (x * x + y * y <= c.radius ** 2)
                best = np.where(hit & (t < best), t, best)
        for axis, value in ((2, 0.0), (2, 3.0), (0, -3.0), (0, 3.0), (1, -3.0), (1, 3.0)):
            t = (value - o[axis]) * inv[:, axis]
            best = np.where((t > 0.0) & (t < best), t, best)
    best = best + g.normal(0.0, 1.0, len(best)) * 0.001 * best ** 2
    return (o[None, :] + best[:, None] * d).astype(np.float32)


def room_cloud(n_surface: int, n_outliers: int, seed: int, n_boxes: int = 20,
               n_cyl: int = 20, size=(0.05, 0.6), noise: float = 0.003) -> np.ndarray:
    """A 6 x 6 x 3 m room: floor and four walls plus `n_boxes` boxes and
    `n_cyl` cylinders inside it.  `n_surface` area-weighted surface points with
    N(0, noise^2) noise, then `n_outliers` points uniform in the room volume.
    float32 [n_surface + n_outliers, 3]."""
    g = _rng(seed)
    R = ROOM
    prims = [
        Plane(2, 0.0, R.copy()),
        Plane(0, 0.0, R.copy()), Plane(0, 6.0, R.copy()),
        Plane(1, 0.0, R.copy()), Plane(1, 6.0, R.copy()),
    ]
    prims += _random_boxes(g, n_boxes, R, *size)
    prims += _random_cylinders(g, n_cyl, R, *size)
    pts = _sample_surfaces(g, prims, n_surface)
    pts = pts + g.normal(0.0, noise, pts.shape)
    out = R[:, 0] + g.random((n_outliers, 3)) * (R[:, 1] - R[:, 0])
    allp = np.concatenate([pts, out], axis=0)
    return allp[g.permutation(len(allp))].astype(np.float32)


# ----------------------------------------------------------------------------
# Robot-like sphere templates and poses
# ----------------------------------------------------------------------------
def chain_template(seed: int, links: int = 6, per_link: int = 10,
                   length=(0.10, 0.25), radius=(0.015, 0.08)) -> np.ndarray:
    """A seeded chain of `links` straight links (lengths uniform in `length`,
    directions uniform on the sphere) with `per_link` sphere centres evenly
    spaced along each link, translated so the centroid is at the origin.
    Radii uniform in `radius`.  float64 [links * per_link, 4]."""
    g = _rng(seed)
    p = np.zeros(3)
    cs = []
    for _ in range(links):
        d = g.normal(size=3)
        d /= np.linalg.norm(d)
        q = p + g.uniform(*length) * d
        for i in range(per_link):
            t = (i + 0.5) / per_link
            cs.append(p + t * (q - p))
        p = q
    cs = np.array(cs)
    cs -= cs.mean(axis=0)
    r = g.uniform(radius[0], radius[1], len(cs))
    return np.concatenate([cs, r[:, None]], axis=1)


def _quat_to_matrix(q: np.ndarray) -> np.ndarray:
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1),
    ], axis=1)


def posed_spheres(template: np.ndarray, n_cfg: int, box, seed: int,
                  chunk: int = 4096) -> np.ndarray:
    """n_cfg rigid poses of `template`: translation uniform in `box`, rotation
    uniform (normalised 4-D Gaussian quaternion).  Centres are R c + t in
    float64, rounded to float32 once.  float32 [n_cfg * len(template), 4],
    configuration-major (the spheres of one pose are consecutive)."""
    box = np.asarray(box, dtype=np.float64)
    g = _rng(seed)
    s = len(template)
    out = np.empty((n_cfg * s, 4), dtype=np.float32)
    c = template[:, :3]
    acc = np.empty((chunk, s))
    tmp = np.empty((chunk, s))
    for a in range(0, n_cfg, chunk):
        b = min(n_cfg, a + chunk)
        k = b - a
        q = g.normal(size=(k, 4))
        q /= np.linalg.norm(q, axis=1, keepdims=True)
        t = box[:, 0] + g.random((k, 3)) * (box[:, 1] - box[:, 0])
        rot = _quat_to_matrix(q)                       # [k, 3, 3]
        blk = out[a * s:b * s].reshape(k, s, 4)
        A, T = acc[:k], tmp[:k]
        for i in range(3):
            # (R[i,0] cx + R[i,1] cy) + R[i,2] cz + t_i, in float64
            np.multiply(rot[:, i, 0:1], c[None, :, 0], out=A)
            np.multiply(rot[:, i, 1:2], c[None, :, 1], out=T)
            A += T
            np.multiply(rot[:, i, 2:3], c[None, :, 2], out=T)
            A += T
            A += t[:, i:i + 1]
            blk[:, :, i] = A
        blk[:, :, 3] = template[None, :, 3]
    return out


def _slerp(q0: np.ndarray, q1: np.ndarray, u: np.ndarray) -> np.ndarray:
    d = np.sum(q0 * q1, axis=1, keepdims=True)
    q1 = np.where(d < 0, -q1, q1)
    d = np.abs(d)
    th = np.arccos(np.clip(d, -1.0, 1.0))
    s = np.sin(th)
    small = s < 1e-9
    a = np.where(small, 1.0 - u, np.sin((1.0 - u) * th) / np.where(small, 1.0, s))
    b = np.where(small, u, np.sin(u * th) / np.where(small, 1.0, s))
    q = a * q0 + b * q1
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def pose_edges(n_edges: int, steps: int, box, seed: int, reach: float = 0.4) -> np.ndarray:
    """Motion edges of a rigid body: each edge runs from a pose (translation
    uniform in `box`, rotation uniform) to a second pose whose translation is
    within `reach` of the first and whose rotation is uniform, in `steps`
    configurations (translation interpolated linearly, rotation by slerp,
    endpoints included when steps > 1).  float64 arithmetic, rounded to float32
    once.  float32 [n_edges * steps, 12]: rotation row-major, then translation."""
    box = np.asarray(box, dtype=np.float64)
    g = _rng(seed)
    q0 = g.normal(size=(n_edges, 4))
    q0 /= np.linalg.norm(q0, axis=1, keepdims=True)
    q1 = g.normal(size=(n_edges, 4))
    q1 /= np.linalg.norm(q1, axis=1, keepdims=True)
    t0 = box[:, 0] + g.random((n_edges, 3)) * (box[:, 1] - box[:, 0])
    t1 = np.clip(t0 + g.uniform(-reach, reach, (n_edges, 3)), box[:, 0], box[:, 1])
    u = (np.arange(steps) / max(steps - 1, 1))[None, :, None]            # [1, steps, 1]
    q = _slerp(np.repeat(q0, steps, 0), np.repeat(q1, steps, 0), np.tile(u[0], (n_edges, 1)))
    t = (t0[:, None, :] * (1.0 - u) + t1[:, None, :] * u).reshape(-1, 3)
    out = np.empty((n_edges * steps, 12), dtype=np.float32)
    out[:, :9] = _quat_to_matrix(q).reshape(-1, 9)
    out[:, 9:] = t
    return out


# ----------------------------------------------------------------------------
# The five workloads
# ----------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    cloud: np.ndarray | list            # float32 [n, 3], or a list of clouds
    spheres: np.ndarray | list           # float32 [m, 4], or one array per cloud
    r_min: float
    r_max: float
    group: int
    r_filter: float | None = None        # Morton filter radius, if the cloud is filtered first
    meta: dict = field(default_factory=dict)


def workload(k: int, scale: float = 1.0) -> Workload:
    """Workload k in 1..5 at full size (scale = 1) or with the query count (and
    for workloads 3 and 5 also the cloud sizes) multiplied by `scale`, for
    quick test runs.  Query counts stay multiples of the group size."""
    if k == 1:
        m = max(1, int(round(100_000 * scale)))
        return Workload("uniform-2k", uniform_cube_cloud(2048, 1001),
                        uniform_spheres(m, [[-0.05, 1.05]] * 3, 0.01, 0.05, 1002),
                        0.01, 0.05, 1)
    if k == 2:
        n_cfg = max(1, int(round(1_000_000 * scale)))
        tpl = chain_template(2003)
        return Workload("tabletop-50k", tabletop_cloud(50_000, 2001),
                        posed_spheres(tpl, n_cfg, WORKSPACE, 2002),
                        0.015, 0.08, 60, r_filter=0.01, meta={"template": tpl})
    if k == 3:
        g = _rng(3000)
        ncl = 64
        sizes = np.rint(np.exp(g.uniform(math.log(1e3), math.log(2e5), ncl))).astype(np.int64)
        qs = (60 * np.rint(np.exp(g.uniform(math.log(1e4), math.log(2e6), ncl)) / 60)).astype(np.int64)
        if scale != 1.0:
            sizes = np.maximum(16, np.rint(sizes * scale)).astype(np.int64)
            qs = np.maximum(60, 60 * np.rint(qs * scale / 60)).astype(np.int64)
        tpl = chain_template(2003)
        clouds = [tabletop_cloud(int(sizes[c]), 3100 + c) for c in range(ncl)]
        sph = [posed_spheres(tpl, int(qs[c]) // 60, WORKSPACE, 3200 + c) for c in range(ncl)]
        return Workload("batched-64", clouds, sph, 0.015, 0.08, 60,
                        meta={"sizes": sizes, "queries": qs, "template": tpl})
    if k == 4:
        m = max(60, int(round(1_000_000 * scale)))
        return Workload("clearance-1M", tabletop_cloud(50_000, 2001),
                        uniform_spheres(m, WORKSPACE, 0.015, 0.08, 4002),
                        0.0, 0.08, 1, r_filter=0.01)
    if k == 5:
        ns = int(round(1_080_000 * min(1.0, scale * 10) if scale != 1.0 else 1_080_000))
        no = int(round(120_000 * min(1.0, scale * 10) if scale != 1.0 else 120_000))
        m = max(1, int(round(100_000_000 * scale)))
        return Workload("room-1.2M", room_cloud(ns, no, 5001),
                        uniform_spheres(m, ROOM, 0.01, 0.1, 5002),
                        0.01, 0.1, 1, r_filter=0.005)
    raise ValueError(f"no workload {k}")
