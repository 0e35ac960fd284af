"""Seeded synthetic inputs for the accessibility-field hot path.

This module only produces *inputs*: scenes, sensor trajectories, LiDAR frames
(via the C ray caster in ``raycast.c``), tool descriptions and orientation sets.
It computes no part of the method itself, so both the CPU oracle and the GPU
library can consume its output without sharing any of the method's arithmetic.

Workloads
---------
``tiny``  sphere (1 m diameter) + 40 cm box with a 3 cm slot, 20 frames x 2,000
          returns, 2 cm voxels, 6 cm truncation, cylinder tool (r 3 cm, 10 cm
          long, 50 cm corridor) at 64 Fibonacci approach directions.
``tree``  procedural 8 m tree (40 cm trunk, 5 branching levels, branch radii
          1-15 cm), 600 frames x 20,000 returns from an orbiting, climbing
          sensor, 1 cm voxels, 4 cm truncation, 30x5x2 cm saw-box tool with a
          1 m corridor at 256 orientations (64 directions x 4 roll angles).

The scan pattern is a Halton sequence over azimuth x elevation that continues
across frames (non-repetitive, Livox Mid-360 style: 360 deg x 59 deg field of
view), as in the paper's synthetic evaluation (Section 4.1).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_raycast.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the ray caster (plain C, OpenMP) into ``synth/_raycast.so``."""
    src = os.path.join(_HERE, "raycast.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", src,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build(force=False)
    lib = ctypes.CDLL(_SO)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.rc_create.restype = ctypes.c_void_p
    lib.rc_create.argtypes = [dp, ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_int,
                              ctypes.c_double]
    lib.rc_destroy.argtypes = [ctypes.c_void_p]
    lib.rc_frame.restype = ctypes.c_long
    lib.rc_frame.argtypes = [ctypes.c_void_p, dp, ctypes.c_double, ctypes.c_double,
                             ctypes.c_uint64, ctypes.c_long, ctypes.c_double,
                             ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double,
                             ctypes.c_long, ctypes.POINTER(ctypes.c_float),
                             ctypes.POINTER(ctypes.c_uint64)]
    lib.rc_cast_many.argtypes = [ctypes.c_void_p, dp, dp, ctypes.c_long,
                                 ctypes.c_double, dp]
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# --------------------------------------------------------------------------
# scenes
# --------------------------------------------------------------------------
@dataclass
class Scene:
    spheres: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))
    boxes: np.ndarray = field(default_factory=lambda: np.zeros((0, 6)))
    capsules: np.ndarray = field(default_factory=lambda: np.zeros((0, 7)))
    cell: float = 0.25

    def caster(self) -> "Caster":
        return Caster(self)


class Caster:
    """Owns a C scene handle."""

    def __init__(self, scene: Scene):
        lib = _load()
        self._lib = lib
        caps = np.ascontiguousarray(scene.capsules, dtype=np.float64).reshape(-1, 7)
        sph = np.ascontiguousarray(scene.spheres, dtype=np.float64).reshape(-1, 4)
        box = np.ascontiguousarray(scene.boxes, dtype=np.float64).reshape(-1, 6)
        self._keep = (caps, sph, box)
        self.h = lib.rc_create(_dptr(caps), len(caps), _dptr(sph), len(sph),
                               _dptr(box), len(box), float(scene.cell))

    def __del__(self):
        if getattr(self, "h", None):
            self._lib.rc_destroy(self.h)
            self.h = None

    def frame(self, origin, el_lo_deg, el_hi_deg, ray0, n_hits, sigma, seed, frame,
              max_range=40.0, max_rays=None):
        o = np.ascontiguousarray(origin, dtype=np.float64)
        out = np.zeros((n_hits, 3), dtype=np.float32)
        used = ctypes.c_uint64(0)
        if max_rays is None:
            max_rays = 400 * n_hits + 100000
        got = self._lib.rc_frame(self.h, _dptr(o), math.radians(el_lo_deg),
                                 math.radians(el_hi_deg), int(ray0), int(n_hits),
                                 float(sigma), int(seed), int(frame), float(max_range),
                                 int(max_rays),
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                 ctypes.byref(used))
        return out[:got], int(used.value)

    def cast(self, origin, dirs, max_range=40.0):
        o = np.ascontiguousarray(origin, dtype=np.float64)
        d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
        t = np.zeros(len(d))
        self._lib.rc_cast_many(self.h, _dptr(o), _dptr(d), len(d), float(max_range),
                               _dptr(t))
        return t


def slotted_box(lo=(0.8, -0.2, 0.0), hi=(1.2, 0.2, 0.4), slot_w=0.03, slot_len=0.30,
                slot_depth=0.20) -> np.ndarray:
    """A solid box with a closed slot cut into its top face, as a union of
    five boxes.  The slot is centred on the box and runs along x, so that a
    sensor on the x axis looks along it."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    cx = 0.5 * (lo[0] + hi[0])
    cy = 0.5 * (lo[1] + hi[1])
    x0, x1 = cx - slot_len / 2, cx + slot_len / 2
    y0, y1 = cy - slot_w / 2, cy + slot_w / 2
    zf = hi[2] - slot_depth
    return np.array([
        [lo[0], lo[1], lo[2], hi[0], y0, hi[2]],
        [lo[0], y1, lo[2], hi[0], hi[1], hi[2]],
        [lo[0], y0, lo[2], hi[0], y1, zf],
        [lo[0], y0, zf, x0, y1, hi[2]],
        [x1, y0, zf, hi[0], y1, hi[2]],
    ])


def tiny_scene() -> Scene:
    """1 m sphere at (0,0,0.5) plus a 40 cm box with a 3 cm-wide, 30 cm-long,
    20 cm-deep slot along x; no ground."""
    return Scene(spheres=np.array([[0.0, 0.0, 0.5, 0.5]]), boxes=slotted_box())


def sphere_scene(radius=0.5, centre=(0.0, 0.0, 0.5)) -> Scene:
    return Scene(spheres=np.array([[*centre, radius]]))


def tree_scene(seed: int = 7, height: float = 8.0, trunk_r: float = 0.20,
               levels: int = 5, r1: float = 0.15, l1: float = 1.6) -> Scene:
    """Procedural tree: tapered trunk (stack of capsules) plus `levels`
    branching levels of capsules.  Each parent carries 3-5 children at a random
    position along it, with a uniform azimuth and 20-70 deg elevation; radius
    halves and length shrinks by ~0.6 per level (15 cm down to ~1 cm)."""
    rng = np.random.default_rng(seed)
    caps = []
    nseg = 8
    for i in range(nseg):
        z0, z1 = height * i / nseg, height * (i + 1) / nseg
        r = trunk_r * (1.0 - 0.75 * (i + 0.5) / nseg)
        caps.append([0.0, 0.0, z0, 0.0, 0.0, z1, r])

    def grow(p0, d, length, radius, level):
        p1 = p0 + d * length
        caps.append([*p0, *p1, radius])
        if level >= levels:
            return
        for _ in range(int(rng.integers(3, 6))):
            s = rng.uniform(0.3, 0.95)
            base = p0 + (p1 - p0) * s
            az = rng.uniform(0.0, 2 * math.pi)
            el = math.radians(rng.uniform(20.0, 70.0))
            cd = np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az),
                           math.sin(el)])
            grow(base, cd, length * 0.6 * rng.uniform(0.85, 1.15), radius * 0.5,
                 level + 1)

    for _ in range(int(rng.integers(3, 6))):
        zb = rng.uniform(0.25, 0.94) * height
        az = rng.uniform(0.0, 2 * math.pi)
        el = math.radians(rng.uniform(20.0, 70.0))
        d = np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az),
                      math.sin(el)])
        grow(np.array([0.0, 0.0, zb]), d, l1 * rng.uniform(0.85, 1.15), r1, 1)
    return Scene(capsules=np.array(caps), cell=0.25)


def box_cluster_scene(seed: int = 11, n_boxes: int = 12, extent: float = 3.0) -> Scene:
    """A cluster of axis-aligned boxes of 10-80 cm on a 20 cm ground slab."""
    rng = np.random.default_rng(seed)
    boxes = [[-extent, -extent, -0.2, extent, extent, 0.0]]
    for _ in range(n_boxes):
        c = rng.uniform(-extent * 0.7, extent * 0.7, size=2)
        s = rng.uniform(0.1, 0.8, size=3)
        z0 = 0.0 if rng.uniform() < 0.7 else rng.uniform(0.2, 1.0)
        boxes.append([c[0] - s[0] / 2, c[1] - s[1] / 2, z0,
                      c[0] + s[0] / 2, c[1] + s[1] / 2, z0 + s[2]])
    return Scene(boxes=np.array(boxes))


# --------------------------------------------------------------------------
# trajectories and frames
# --------------------------------------------------------------------------
def circle_poses(n: int, radius: float = 3.0, centre=(0.5, 0.0), z: float = 1.5):
    a = 2 * math.pi * np.arange(n) / n
    return np.stack([centre[0] + radius * np.cos(a), centre[1] + radius * np.sin(a),
                     np.full(n, z)], axis=1)


def orbit_poses(n: int, seed: int = 3, r_lo: float = 4.0, r_hi: float = 6.0,
                z_lo: float = 0.5, z_hi: float = 8.0, period: int = 150, span: int = 600):
    """Seeded orbit around the z axis: radius wanders in [r_lo, r_hi], altitude
    climbs from z_lo to z_hi and back once every `span` frames, small jitter."""
    rng = np.random.default_rng(seed)
    t = np.arange(n, dtype=np.float64)
    ph = rng.uniform(0, 2 * math.pi, size=3)
    ang = 2 * math.pi * t / period + ph[0]
    rad = 0.5 * (r_lo + r_hi) + 0.5 * (r_hi - r_lo) * np.sin(2 * math.pi * t / (2.3 * period) + ph[1])
    frac = 0.5 - 0.5 * np.cos(2 * math.pi * t / span)
    z = z_lo + (z_hi - z_lo) * frac
    jit = rng.normal(0.0, 0.03, size=(n, 3))
    return np.stack([rad * np.cos(ang), rad * np.sin(ang), z], axis=1) + jit


@dataclass
class Frame:
    xyz: np.ndarray      # float32 [n, 3], world frame
    origin: np.ndarray   # float32 [3], sensor position for the frame
    frame_id: int


def make_frames(scene: Scene, poses, n_hits, sigma: float, seed: int,
                el_lo: float, el_hi: float, max_range: float = 40.0):
    """One frame per pose; `n_hits` is an int or a per-frame sequence.  The
    Halton index continues across frames."""
    caster = scene.caster()
    frames = []
    ray0 = 0
    for i, p in enumerate(np.asarray(poses)):
        o32 = np.asarray(p, dtype=np.float32)
        nh = int(n_hits if np.isscalar(n_hits) else n_hits[i])
        xyz, used = caster.frame(o32.astype(np.float64), el_lo, el_hi, ray0, nh, sigma,
                                 seed, i, max_range=max_range)
        ray0 += used
        frames.append(Frame(np.ascontiguousarray(xyz), o32, i))
    return frames


# --------------------------------------------------------------------------
# tools and orientations
# --------------------------------------------------------------------------
CYLINDER = 0
BOX = 1


@dataclass
class Tool:
    """Tool solid in its local frame: approach axis +x, tip at the origin.
    Body: 0 <= x <= length; corridor: length < x <= length + corridor; both
    with the same cross-section (disc of `radius`, or width x height box).
    Points closer than `r_s` to the tip are excluded (self-exclusion)."""
    shape: int
    length: float
    corridor: float
    r_s: float
    radius: float = 0.0
    width: float = 0.0
    height: float = 0.0


def cylinder_tool(radius=0.03, length=0.10, corridor=0.50) -> Tool:
    return Tool(CYLINDER, length, corridor, r_s=radius, radius=radius)


def box_tool(length=0.30, width=0.05, height=0.02, corridor=1.0) -> Tool:
    return Tool(BOX, length, corridor, r_s=math.hypot(width / 2, height / 2),
                width=width, height=height)


def tool_samples(tool: Tool, n_stations: int = 16) -> np.ndarray:
    """Points of the tool solid in its local frame (approach axis +x, tip at
    the origin) for the smoothed score: `n_stations` stations evenly spaced
    from r_s to length + corridor, and at each the four rim points of the
    cross-section (cylinder: radius at 0, 90, 180, 270 degrees; box: the
    corners).  float32, (4 n_stations) x 3."""
    xs = np.linspace(tool.r_s, tool.length + tool.corridor, n_stations)
    if tool.shape == CYLINDER:
        rim = [(tool.radius, 0.0), (0.0, tool.radius), (-tool.radius, 0.0), (0.0, -tool.radius)]
    else:
        hw, hh = tool.width / 2, tool.height / 2
        rim = [(hw, hh), (-hw, hh), (-hw, -hh), (hw, -hh)]
    return np.array([[x, y, z] for x in xs for y, z in rim], np.float32)


def pencil_points(tip_length=0.04, radius=0.02, length=0.12, corridor=0.40,
                  spacing=0.005):
    """A pencil-shaped tool as point samples of its 3D model in its local
    frame (approach axis +x, tip at the origin): a cone from the tip to a
    disc of `radius` at x = tip_length, then a cylindrical shaft to x =
    length (the body), then the approach corridor of the shaft's
    cross-section to x = length + corridor.  Samples lie on a regular grid of
    `spacing` inside each solid.  Returns (body [M, 3], corridor [N, 3]),
    float64."""
    r = np.arange(-radius, radius + 1e-12, spacing)
    yz = np.array([(y, z) for y in r for z in r if y * y + z * z <= radius * radius + 1e-12])
    body, far = [], []
    for x in np.arange(0.0, length + corridor + 1e-12, spacing):
        rad = radius * min(1.0, x / tip_length)
        sel = yz[(yz ** 2).sum(1) <= rad * rad + 1e-12]
        pts = np.column_stack([np.full(len(sel), x), sel])
        (body if x <= length + 1e-12 else far).append(pts)
    return np.concatenate(body), np.concatenate(far)


def quaternion_towards(dirs: np.ndarray) -> np.ndarray:
    """Unit quaternions (w, x, y, z) of the shortest rotations taking the
    tool axis +x to each direction (the antipode turns about +z)."""
    out = []
    for d in np.asarray(dirs, dtype=np.float64):
        d = d / np.linalg.norm(d)
        w = 1.0 + d[0]
        if w < 1e-9:
            out.append([0.0, 0.0, 0.0, 1.0])
            continue
        q = np.array([w, 0.0, -d[2], d[1]])   # (1 + e_x.d, e_x x d)
        out.append(q / np.linalg.norm(q))
    return np.array(out, np.float32)


def fibonacci_directions(n: int) -> np.ndarray:
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - (2 * k + 1) / n
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def yaw_directions(n: int = 180) -> np.ndarray:
    """The paper's yaw-only candidate set (horizontal approach)."""
    a = 2 * math.pi * np.arange(n) / n
    return np.stack([np.cos(a), np.sin(a), np.zeros(n)], axis=1)


def orientations(dirs: np.ndarray, n_roll: int = 1) -> np.ndarray:
    """Rotation matrices (K x 9, row-major) whose columns are the tool's local
    axes in world coordinates: column 0 is the approach direction, columns 1-2
    span the cross-section, rolled by r*pi/n_roll.  Orientation k = dir*n_roll
    + roll."""
    out = []
    for d in np.asarray(dirs, dtype=np.float64):
        e1 = d / np.linalg.norm(d)
        a = np.array([0.0, 0.0, 1.0]) if abs(e1[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
        e2 = np.cross(a, e1)
        e2 /= np.linalg.norm(e2)
        e3 = np.cross(e1, e2)
        for r in range(n_roll):
            ph = r * math.pi / n_roll
            c, s = math.cos(ph), math.sin(ph)
            f2 = c * e2 + s * e3
            f3 = -s * e2 + c * e3
            out.append(np.stack([e1, f2, f3], axis=1).reshape(9))
    return np.ascontiguousarray(np.array(out, dtype=np.float64))


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    voxel: float
    trunc: float
    r_c: float
    scene: Scene
    poses: np.ndarray
    n_hits: object
    sigma: float
    seed: int
    el_lo: float
    el_hi: float
    tool: Tool
    rot: np.ndarray
    n_frames: int

    def frames(self, n: int | None = None):
        n = self.n_frames if n is None else n
        nh = self.n_hits if np.isscalar(self.n_hits) else list(self.n_hits)[:n]
        return make_frames(self.scene, self.poses[:n], nh, self.sigma, self.seed,
                           self.el_lo, self.el_hi)


def tiny(sigma: float = 0.01, seed: int = 1, scene: Scene | None = None,
         n_frames: int = 20, n_hits: int = 2000) -> Workload:
    """Sphere + slotted box, 20 x 2,000 returns, v = 2 cm, tau = 6 cm.  The
    sensor is mounted inverted (elevation -52..+7 deg) on a 3 m circle at
    1.5 m so that it looks down onto the objects."""
    return Workload("tiny", 0.02, 0.06, 0.01, scene or tiny_scene(),
                    circle_poses(n_frames), n_hits, sigma, seed, -52.0, 7.0,
                    cylinder_tool(), orientations(fibonacci_directions(64), 1),
                    n_frames)


def tree(n_frames: int = 600, n_hits=20000, sigma: float = 0.02, seed: int = 5,
         tree_seed: int = 7, traj_seed: int = 3) -> Workload:
    """Procedural 8 m tree, 600 x 20,000 returns, v = 1 cm, tau = 4 cm, saw box
    30x5x2 cm with 1 m corridor at 64 directions x 4 rolls."""
    poses = orbit_poses(max(600, n_frames), seed=traj_seed)
    return Workload("tree", 0.01, 0.04, 0.01, tree_scene(tree_seed), poses, n_hits,
                    sigma, seed, -7.0, 52.0, box_tool(),
                    orientations(fibonacci_directions(64), 4), n_frames)


def window_walk(n_frames: int = 48, n_hits: int = 3000, sigma: float = 0.01, seed: int = 17,
                scene_seed: int = 11) -> Workload:
    """Sliding-window workload: a 6 x 6 m box cluster on a ground slab, the
    sensor on a 2 m circle at 1.2 m looking down (elevation -52..+7 deg), one
    lap in `n_frames` frames (26 cm per frame at 48), v = 2 cm, tau = 6 cm.
    With a 3.2 m window (20 blocks) the window shifts every few frames and
    regions leave it and come back within the lap."""
    return Workload("window_walk", 0.02, 0.06, 0.01, box_cluster_scene(scene_seed),
                    circle_poses(n_frames, radius=2.0, centre=(0.0, 0.0), z=1.2), n_hits,
                    sigma, seed, -52.0, 7.0, cylinder_tool(),
                    orientations(fibonacci_directions(64), 1), n_frames)


def uneven_counts(n: int, lo: int = 5000, hi: int = 40000, seed: int = 9):
    return np.random.default_rng(seed).integers(lo, hi + 1, size=n)


def batch_tools(seed: int = 13):
    """Eight seeded tools for the batching workload: cylinders (even index)
    and boxes (odd) with 2-8 cm cross-sections, 10-30 cm bodies and
    0.3-1.5 m corridors."""
    rng = np.random.default_rng(seed)
    tools = []
    for i in range(8):
        size = float(rng.uniform(0.02, 0.08))
        length = float(rng.uniform(0.10, 0.30))
        corridor = float(rng.uniform(0.3, 1.5))
        if i % 2 == 0:
            tools.append(cylinder_tool(radius=size / 2, length=length, corridor=corridor))
        else:
            height = float(rng.uniform(0.02, size))
            tools.append(box_tool(length=length, width=size, height=height, corridor=corridor))
    return tools


def batch(n_frames: int = 600, seed: int = 5, counts_seed: int = 9) -> Workload:
    """The tree scene with frames of 5,000-40,000 returns (uniform, seeded);
    the tools and their 512 orientations (128 directions x 4 rolls) come from
    batch_tools() and orientations(fibonacci_directions(128), 4)."""
    w = tree(n_frames=n_frames, seed=seed)
    w.name = "batch"
    w.n_hits = uneven_counts(max(600, n_frames), seed=counts_seed)
    w.rot = orientations(fibonacci_directions(128), 4)
    return w


@dataclass
class ServeStream:
    workload: Workload
    phase: float   # seconds after the start at which the stream's first frame arrives


def serving(n_streams: int = 4, n_frames: int = 600, seed: int = 21):
    """Concurrent sensor streams: even streams see a seeded tree, odd streams a
    seeded box cluster; each has its own trajectory, its own tool (from
    batch_tools()) at 256 orientations (64 directions x 4 rolls), frames of
    5,000-40,000 returns (uniform, seeded) at 10 Hz from a seeded phase;
    v = 1 cm, tau = 4 cm."""
    rng = np.random.default_rng(seed)
    tools = batch_tools()
    rot = orientations(fibonacci_directions(64), 4)
    out = []
    for s in range(n_streams):
        if s % 2 == 0:
            scene = tree_scene(seed=7 + s)
            poses = orbit_poses(max(600, n_frames), seed=3 + s)
        else:
            scene = box_cluster_scene(seed=11 + s)
            poses = orbit_poses(max(600, n_frames), seed=3 + s, r_lo=3.5, r_hi=5.0,
                                z_lo=0.5, z_hi=3.0)
        w = Workload("serve%d" % s, 0.01, 0.04, 0.01, scene, poses,
                     uneven_counts(max(600, n_frames), seed=9 + s), 0.02, 5 + s, -7.0, 52.0,
                     tools[s % len(tools)], rot, n_frames)
        out.append(ServeStream(w, float(rng.uniform(0.0, 0.1))))
    return out
