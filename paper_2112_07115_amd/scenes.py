"""Seeded synthetic scenes for the dynamic vehicular ray tracer.

This module only builds inputs: triangle geometry, materials, transmitter and
receiver positions, per-frame rigid transforms of the moving vehicles and
(optionally) random ray directions.  It holds none of the propagation
arithmetic, so both the HIP library and the CPU oracle can be fed from it.

The paper evaluates on a commercial European-town model and an indoor office
(Sec. III, Sec. IV) that are not available here; the scenes below stand in for
its "typical vehicular communication scenario" (Sec. IV-A): an urban street grid
with box buildings on a ground plane and box-shaped vehicles moving along lanes.
The material table follows the paper's choice of one reflection property per
object class (Table II), expressed as relative permittivity and conductivity.

Arrays use float32 for geometry (the library traces in FP32) and float64 for
material constants.  Every scene is a pure function of its seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

# material rows: (eps_r, sigma [S/m], const_gamma); const_gamma = NaN selects Fresnel
CONCRETE = (5.31, 0.48, float("nan"))
# Table II's materials as constant-magnitude reflectors, with their
# penetration losses (dB; inf: not penetrable)
WALL_OUTDOOR = (5.31, 0.48, 0.8)
WALL_INDOOR = (5.31, 0.48, 0.7)
GLASS_INDOOR = (6.27, 0.0, 0.74)
PEN_WALL_INDOOR_DB = 20.0
PEN_GLASS_INDOOR_DB = 5.0
GROUND = (15.0, 0.035, float("nan"))
METAL = (1.0, 1.0e7, float("nan"))


@dataclass
class Scene:
    name: str
    vertices: np.ndarray            # f32 [Nv, 3], upload (reference) pose
    tris: np.ndarray                # i32 [Nt, 3]
    tri_face: np.ndarray            # i32 [Nt]
    face_material: np.ndarray       # i32 [Nf]
    face_object: np.ndarray         # i32 [Nf], -1 = static
    materials: np.ndarray           # f64 [Nm, 3] (eps_r, sigma, const_gamma)
    object_vertex_range: np.ndarray  # i64 [No, 2], half-open vertex ranges
    tx: np.ndarray                  # f32 [Ntx, 3]
    rx: np.ndarray                  # f32 [Nrx, 3]
    rx_radius: float = 0.5
    n_rays: int = 4096
    max_reflections: int = 2
    freqs_hz: List[float] = field(default_factory=lambda: [28e9])
    tx_power_w: float = 5.0
    n_frames: int = 1
    dt: float = 0.1
    # frame -> f32 [No, 3, 4] object-to-world transforms relative to the upload pose
    transforms_fn: Optional[Callable[[int], np.ndarray]] = None
    # frame -> f32 [Nrx, 3] receiver positions (moving receivers); None: rx at every frame
    rx_fn: Optional[Callable[[int], np.ndarray]] = None
    # penetration loss per material in dB (+inf: opaque; Table II), and the
    # transmissions a path may have (0: no penetration, the outdoor setting)
    penetration_db: Optional[np.ndarray] = None
    max_transmissions: int = 0

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])

    @property
    def n_faces(self) -> int:
        return int(self.face_material.shape[0])

    @property
    def n_objects(self) -> int:
        return int(self.object_vertex_range.shape[0])

    def transforms(self, frame: int) -> np.ndarray:
        if self.transforms_fn is None or self.n_objects == 0:
            return identity_transforms(self.n_objects)
        return self.transforms_fn(frame)

    def rx_at(self, frame: int) -> np.ndarray:
        """Receiver positions at a frame (vehicle-mounted receivers move)."""
        return self.rx if self.rx_fn is None else self.rx_fn(frame)


def identity_transforms(n: int) -> np.ndarray:
    xf = np.zeros((n, 3, 4), dtype=np.float32)
    xf[:, 0, 0] = 1.0
    xf[:, 1, 1] = 1.0
    xf[:, 2, 2] = 1.0
    return xf


class _MeshBuilder:
    """Accumulates shared-vertex meshes whose triangles are grouped in planar faces."""

    def __init__(self):
        self.verts: List[np.ndarray] = []
        self.tris: List[np.ndarray] = []
        self.tri_face: List[np.ndarray] = []
        self.face_material: List[int] = []
        self.face_object: List[int] = []
        self.nv = 0
        self.object_ranges: List[tuple] = []

    def add_box(self, lo, hi, cells, material: int, obj: int = -1) -> None:
        """Axis-aligned box [lo, hi] tessellated into cells=(nx, ny, nz) lattice quads.

        The six sides are six faces (-x, +x, -y, +y, -z, +z); lattice points are
        shared between sides so the mesh is closed.
        """
        nx, ny, nz = cells
        lo = np.asarray(lo, dtype=np.float64)
        hi = np.asarray(hi, dtype=np.float64)
        index = {}
        pts = []

        def vid(i, j, k):
            key = (i, j, k)
            if key not in index:
                index[key] = len(pts)
                pts.append((lo[0] + (hi[0] - lo[0]) * i / nx,
                            lo[1] + (hi[1] - lo[1]) * j / ny,
                            lo[2] + (hi[2] - lo[2]) * k / nz))
            return index[key]

        tris = []
        fids = []
        base_face = len(self.face_material)
        # (fixed axis, fixed value index, axis a, count a, axis b, count b)
        sides = [
            (0, 0, 1, ny, 2, nz), (0, nx, 1, ny, 2, nz),
            (1, 0, 0, nx, 2, nz), (1, ny, 0, nx, 2, nz),
            (2, 0, 0, nx, 1, ny), (2, nz, 0, nx, 1, ny),
        ]
        for f, (ax, fixed, a, na, b, nb) in enumerate(sides):
            for ia in range(na):
                for ib in range(nb):
                    quad = []
                    for (da, db) in ((0, 0), (1, 0), (1, 1), (0, 1)):
                        c = [0, 0, 0]
                        c[ax] = fixed
                        c[a] = ia + da
                        c[b] = ib + db
                        quad.append(vid(*c))
                    tris.append((quad[0], quad[1], quad[2]))
                    tris.append((quad[0], quad[2], quad[3]))
                    fids += [base_face + f, base_face + f]
            self.face_material.append(material)
            self.face_object.append(obj)
        v0 = self.nv
        self.verts.append(np.asarray(pts, dtype=np.float64).astype(np.float32))
        self.tris.append(np.asarray(tris, dtype=np.int64) + v0)
        self.tri_face.append(np.asarray(fids, dtype=np.int64))
        self.nv += len(pts)
        if obj >= 0:
            self.object_ranges.append((v0, self.nv))

    def add_ground(self, half: float, material: int) -> None:
        pts = np.array([[-half, -half, 0.0], [half, -half, 0.0],
                        [half, half, 0.0], [-half, half, 0.0]], dtype=np.float32)
        f = len(self.face_material)
        v0 = self.nv
        self.verts.append(pts)
        self.tris.append(np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int64) + v0)
        self.tri_face.append(np.array([f, f], dtype=np.int64))
        self.face_material.append(material)
        self.face_object.append(-1)
        self.nv += 4

    def add_polygon_face(self, pts, tris, material: int) -> None:
        """One planar face given explicitly (used by the small closed-form scenes)."""
        pts = np.asarray(pts, dtype=np.float32)
        f = len(self.face_material)
        v0 = self.nv
        self.verts.append(pts)
        self.tris.append(np.asarray(tris, dtype=np.int64) + v0)
        self.tri_face.append(np.full(len(tris), f, dtype=np.int64))
        self.face_material.append(material)
        self.face_object.append(-1)
        self.nv += len(pts)

    def add_faces(self, faces, material, obj: int = -1) -> None:
        """Planar faces given as (points [n][3], triangles [m][3] local to
        the points), with contiguous vertices; obj >= 0 makes them one moving
        object."""
        v0 = self.nv
        for pts, tris in faces:
            pts = np.asarray(pts, dtype=np.float64).astype(np.float32)
            f = len(self.face_material)
            base = self.nv
            self.verts.append(pts)
            self.tris.append(np.asarray(tris, dtype=np.int64) + base)
            self.tri_face.append(np.full(len(tris), f, dtype=np.int64))
            self.face_material.append(material)
            self.face_object.append(obj)
            self.nv += len(pts)
        if obj >= 0:
            self.object_ranges.append((v0, self.nv))

    def finish(self, name, materials, tx, rx, **kw) -> Scene:
        return Scene(
            name=name,
            vertices=np.concatenate(self.verts).astype(np.float32) if self.verts
            else np.zeros((0, 3), np.float32),
            tris=np.concatenate(self.tris).astype(np.int32) if self.tris
            else np.zeros((0, 3), np.int32),
            tri_face=np.concatenate(self.tri_face).astype(np.int32) if self.tri_face
            else np.zeros((0,), np.int32),
            face_material=np.asarray(self.face_material, dtype=np.int32),
            face_object=np.asarray(self.face_object, dtype=np.int32),
            materials=np.asarray(materials, dtype=np.float64).reshape(-1, 3),
            object_vertex_range=np.asarray(self.object_ranges, dtype=np.int64).reshape(-1, 2),
            tx=np.asarray(tx, dtype=np.float32).reshape(-1, 3),
            rx=np.asarray(rx, dtype=np.float32).reshape(-1, 3),
            **kw,
        )


def static_toy(seed: int = 1) -> Scene:
    """Static toy scene, one frame: 200 m ground, 4 random boxes, 16 receivers.

    Ground [-100, 100]^2 (2 triangles, ground material); four axis-aligned
    concrete boxes with footprints U(20, 40) m per side, heights U(10, 30) m and
    centres U(-80, 80)^2, rejection-sampled to keep 1 m clear of each other, of
    the transmitter and of every receiver.  Tx at (0, 0, 5); receivers on the
    grid {-75, -25, 25, 75}^2 at 1.5 m with 0.5 m capture spheres; 4096 rays,
    2 reflections, 28 GHz, 5 W (the paper's outdoor transmit power, Sec. III).
    """
    rng = np.random.default_rng(seed)
    tx = np.array([[0.0, 0.0, 5.0]])
    g = np.array([-75.0, -25.0, 25.0, 75.0])
    rx = np.array([[x, y, 1.5] for x in g for y in g])
    boxes = []
    while len(boxes) < 4:
        sx, sy = rng.uniform(20.0, 40.0, size=2)
        h = rng.uniform(10.0, 30.0)
        cx, cy = rng.uniform(-80.0, 80.0, size=2)
        lo = np.array([cx - sx / 2, cy - sy / 2])
        hi = np.array([cx + sx / 2, cy + sy / 2])
        ok = True
        for (blo, bhi, _) in boxes:
            if np.all(lo - 1.0 < bhi) and np.all(blo < hi + 1.0):
                ok = False
        for p in np.concatenate([tx[:, :2], rx[:, :2]]):
            if np.all(p > lo - 1.0) and np.all(p < hi + 1.0):
                ok = False
        if ok:
            boxes.append((lo, hi, h))
    mb = _MeshBuilder()
    mb.add_ground(100.0, material=1)
    for (lo, hi, h) in boxes:
        mb.add_box((lo[0], lo[1], 0.0), (hi[0], hi[1], h), (1, 1, 1), material=0)
    return mb.finish("static_toy", [CONCRETE, GROUND], tx, rx,
                     rx_radius=0.5, n_rays=4096, max_reflections=2,
                     freqs_hz=[28e9], tx_power_w=5.0, n_frames=1)


# ---- dynamic urban grid -------------------------------------------------------

GRID_BLOCKS = 8
BLOCK = 40.0
STREET = 15.0
EXTENT = GRID_BLOCKS * BLOCK + (GRID_BLOCKS + 1) * STREET   # 455 m
HALF = EXTENT / 2.0                                          # 227.5 m
LANE_OFFSET = 2.25
VEHICLE = (4.5, 1.8, 1.5)
VEHICLE_CLEARANCE = 0.3


def _block_origin(i: int) -> float:
    return -HALF + STREET + i * (BLOCK + STREET)


def _street_centre(k: int) -> float:
    return -HALF + STREET / 2.0 + k * (BLOCK + STREET)


# Building material classes of the eight-class urban variant (the
# calibration workload): (eps_r, sigma [S/m]) starting values of plausible
# facade materials; the classes are what a fit tells apart.
FACADE_CLASSES = [(5.31, 0.48), (3.75, 0.04), (6.5, 0.3), (4.0, 0.1), (2.5, 0.01), (7.0, 0.2)]


def dynamic_urban(seed: int = 2, n_vehicles: int = 40, n_rx: int = 256,
                  n_rays: int = 1 << 20, max_reflections: int = 4,
                  n_frames: int = 60, material_classes: int = 3) -> Scene:
    """Dynamic urban scene: 8x8 Manhattan grid, moving metal vehicles, 60 frames at 10 Hz.

    material_classes = 3: concrete buildings, ground, metal vehicles
    (materials 0, 1, 2).  material_classes = 8: six facade classes for the
    buildings (block (i, j) gets class (i + 2 j) mod 6), ground 6, vehicles 7.

    Blocks of 40 m separated by 15 m streets (border streets included, 455 m
    across, centred on the origin) on a [-260, 260]^2 ground plane.  One
    concrete box building per block, footprint 40x40 m, height U(10, 60) m,
    tessellated 3x3x6.  Each vehicle is a 4.5x1.8x1.5 m metal box 0.3 m above
    the ground, tessellated 12x5x4 (512 triangles), placed on one of 18 streets
    and one of its two lanes (+-2.25 m from the centre line) at a uniform
    position, moving at U(10, 20) m/s in the lane direction, wrapping
    periodically at the grid edge and passing through intersections.  The
    transmitter is a rooftop base station: a 2 m mast (the paper's transmitter
    height) at the roof corner of block (3, 3) that faces the central
    intersection, 0.5 m inside both roof edges (a mast at the roof centre is
    shadowed by its own roof).  Receivers are uniform on the sidewalks
    (4.5-7.0 m from a street centre line, away from intersections) at 1.5 m.
    """
    rng = np.random.default_rng(seed)
    heights = rng.uniform(10.0, 60.0, size=(GRID_BLOCKS, GRID_BLOCKS))
    mb = _MeshBuilder()
    assert material_classes in (3, 8)
    eight = material_classes == 8
    mat_ground, mat_vehicle = (6, 7) if eight else (1, 2)
    mb.add_ground(260.0, material=mat_ground)
    for i in range(GRID_BLOCKS):
        for j in range(GRID_BLOCKS):
            x0, y0 = _block_origin(i), _block_origin(j)
            mb.add_box((x0, y0, 0.0), (x0 + BLOCK, y0 + BLOCK, heights[i, j]),
                       (3, 3, 6), material=(i + 2 * j) % 6 if eight else 0)
    # rooftop base station: a 2 m mast (the paper's transmitter height) 0.5 m
    # inside the roof corner of block (3, 3) that faces the central intersection
    corner = _block_origin(3) + BLOCK - 0.5
    tx = np.array([[corner, corner, heights[3, 3] + 2.0]])

    # vehicles: (axis along which it moves, lane coordinate, direction, start, speed)
    veh = []
    for v in range(n_vehicles):
        street = int(rng.integers(0, 2 * (GRID_BLOCKS + 1)))
        lane = int(rng.integers(0, 2))
        u = rng.uniform(-HALF, HALF)
        speed = rng.uniform(10.0, 20.0)
        k = street % (GRID_BLOCKS + 1)
        c = _street_centre(k)
        if street <= GRID_BLOCKS:      # street running along x at y = c
            axis = 0
            lane_c = c - LANE_OFFSET if lane == 0 else c + LANE_OFFSET
            direction = 1.0 if lane == 0 else -1.0
        else:                          # street running along y at x = c
            axis = 1
            lane_c = c + LANE_OFFSET if lane == 0 else c - LANE_OFFSET
            direction = 1.0 if lane == 0 else -1.0
        veh.append((axis, lane_c, direction, u, speed))
        L, W, H = VEHICLE
        if axis == 0:
            lo = (u - L / 2, lane_c - W / 2, VEHICLE_CLEARANCE)
            hi = (u + L / 2, lane_c + W / 2, VEHICLE_CLEARANCE + H)
            cells = (12, 5, 4)
        else:
            lo = (lane_c - W / 2, u - L / 2, VEHICLE_CLEARANCE)
            hi = (lane_c + W / 2, u + L / 2, VEHICLE_CLEARANCE + H)
            cells = (5, 12, 4)
        mb.add_box(lo, hi, cells, material=mat_vehicle, obj=v)

    centres = np.array([_street_centre(k) for k in range(GRID_BLOCKS + 1)])
    rx = []
    while len(rx) < n_rx:
        street = int(rng.integers(0, 2 * (GRID_BLOCKS + 1)))
        side = 1.0 if rng.integers(0, 2) == 1 else -1.0
        off = rng.uniform(4.5, 7.0)
        along = rng.uniform(-HALF + 2.5, HALF - 2.5)
        if np.any(np.abs(along - centres) < STREET / 2 + 0.5):
            continue   # keep receivers out of intersections, where cross traffic passes
        c = centres[street % (GRID_BLOCKS + 1)]
        if street <= GRID_BLOCKS:
            rx.append((along, c + side * off, 1.5))
        else:
            rx.append((c + side * off, along, 1.5))

    dt = 0.1
    veh_arr = veh

    def transforms(frame: int) -> np.ndarray:
        xf = identity_transforms(len(veh_arr))
        for v, (axis, _lane_c, direction, u, speed) in enumerate(veh_arr):
            p = u + direction * speed * frame * dt
            p = -HALF + np.mod(p + HALF, EXTENT)
            xf[v, axis, 3] = np.float32(p - u)
        return xf

    mats = ([(e, sg, float("nan")) for e, sg in FACADE_CLASSES] + [GROUND, METAL]) if eight \
        else [CONCRETE, GROUND, METAL]
    return mb.finish("dynamic_urban", mats, tx, np.array(rx),
                     rx_radius=0.5, n_rays=n_rays, max_reflections=max_reflections,
                     freqs_hz=[28e9], tx_power_w=5.0, n_frames=n_frames, dt=dt,
                     transforms_fn=transforms)


# ---- small scenes with closed-form answers -------------------------------------

def free_space(tx, rx, **kw) -> Scene:
    """No geometry at all: only the direct path exists."""
    mb = _MeshBuilder()
    return mb.finish("free_space", [CONCRETE], tx, rx, **kw)


def ground_only(tx, rx, material=GROUND, half: float = 2000.0, **kw) -> Scene:
    """A single ground plane z = 0 (two triangles)."""
    mb = _MeshBuilder()
    mb.add_ground(half, material=0)
    return mb.finish("ground_only", [material], tx, rx, **kw)


def single_wall(tx, rx, x: float = 10.0, half: float = 500.0, material=CONCRETE, **kw) -> Scene:
    """One vertical wall in the plane x = const, spanning |y|, |z| <= half."""
    mb = _MeshBuilder()
    pts = [[x, -half, -half], [x, half, -half], [x, half, half], [x, -half, half]]
    mb.add_polygon_face(pts, [[0, 1, 2], [0, 2, 3]], material=0)
    return mb.finish("single_wall", [material], tx, rx, **kw)


def corner(tx, rx, half: float = 200.0, material=CONCRETE, **kw) -> Scene:
    """Two perpendicular walls x = 0 (y >= 0) and y = 0 (x >= 0), both |z| <= half."""
    mb = _MeshBuilder()
    mb.add_polygon_face([[0, 0, -half], [0, half, -half], [0, half, half], [0, 0, half]],
                        [[0, 1, 2], [0, 2, 3]], material=0)
    mb.add_polygon_face([[0, 0, -half], [half, 0, -half], [half, 0, half], [0, 0, half]],
                        [[0, 1, 2], [0, 2, 3]], material=0)
    return mb.finish("corner", [material], tx, rx, **kw)


def parallel_walls(tx, rx, x0: float = -10.0, x1: float = 10.0, half: float = 500.0,
                   material=CONCRETE, **kw) -> Scene:
    """Two facing walls x = x0 and x = x1 (a street canyon without ground)."""
    mb = _MeshBuilder()
    for x in (x0, x1):
        mb.add_polygon_face([[x, -half, -half], [x, half, -half], [x, half, half], [x, -half, half]],
                            [[0, 1, 2], [0, 2, 3]], material=0)
    return mb.finish("parallel_walls", [material], tx, rx, **kw)


def slabs(tx, rx, walls, materials, penetration_db, half: float = 60.0, max_transmissions: int = 2,
          **kw) -> Scene:
    """Parallel planar walls x = x_i (one face each, |y|, |z| <= half) of the
    given materials, for closed-form transmission checks."""
    mb = _MeshBuilder()
    for x, m in walls:
        mb.add_polygon_face([[x, -half, -half], [x, half, -half], [x, half, half], [x, -half, half]],
                            [[0, 1, 2], [0, 2, 3]], m)
    return mb.finish("slabs", materials, tx, rx, penetration_db=np.asarray(penetration_db, np.float64),
                     max_transmissions=max_transmissions, **kw)


def _wall_cells(mb, axis: int, pos: float, span, zs, kind, mats) -> None:
    """A vertical wall in the plane x = pos (axis 0) or y = pos (axis 1), cut
    into cells along `span` (breakpoints along the other horizontal axis) and
    `zs` (heights); kind(i, j) gives cell (i, j)'s material key, None for an
    opening.  Cells of one material form one face."""
    groups = {}
    for i in range(len(span) - 1):
        for j in range(len(zs) - 1):
            k = kind(i, j)
            if k is None:
                continue
            groups.setdefault(k, []).append((span[i], span[i + 1], zs[j], zs[j + 1]))
    for k, cells in groups.items():
        pts, tris = [], []
        for (a0, a1, z0, z1) in cells:
            q = [(a0, z0), (a1, z0), (a1, z1), (a0, z1)]
            base = len(pts)
            for (a, z) in q:
                pts.append([pos, a, z] if axis == 0 else [a, pos, z])
            tris += [[base, base + 1, base + 2], [base, base + 2, base + 3]]
        mb.add_polygon_face(pts, tris, mats[k])


def indoor_office(n_rays: int = 1 << 18, max_reflections: int = 2, max_transmissions: int = 2,
                  rx_step: float = 1.0) -> Scene:
    """An office floor (Sec. III's indoor setting: walls, doors and windows of
    Table II's materials, a 2 m high transmitter, 30 GHz, 0.5 W).

    24 m x 14 m x 3 m: concrete floor and ceiling and outdoor walls (opaque), a
    corridor between y = 6 and y = 8 whose walls (indoor walls, 20 dB) have a
    door opening and a glass window (5 dB) per room, and partitions at x = 6,
    12 and 18 with a glass window each.  Receivers on a rx_step grid at
    1.5 m; the transmitter in the corridor.  Constant-magnitude reflection
    coefficients of Table II (0.8, 0.7, 0.74) for the walls and the glass."""
    mb = _MeshBuilder()
    mats = {"concrete": 0, "outdoor": 1, "wall": 2, "glass": 3}
    W, D, H = 24.0, 14.0, 3.0
    mb.add_polygon_face([[0, 0, 0], [W, 0, 0], [W, D, 0], [0, D, 0]], [[0, 1, 2], [0, 2, 3]], mats["concrete"])
    mb.add_polygon_face([[0, 0, H], [W, 0, H], [W, D, H], [0, D, H]], [[0, 1, 2], [0, 2, 3]], mats["concrete"])
    for axis, pos, length in ((0, 0.0, D), (0, W, D), (1, 0.0, W), (1, D, W)):
        _wall_cells(mb, axis, pos, [0.0, length], [0.0, H], lambda i, j: "outdoor", mats)
    # corridor walls: per 6 m room a door (x in [2.5, 3.5], below 2.1 m) and
    # a window (x in [4.0, 5.5], 1.0 to 2.2 m)
    xs = sorted({0.0, W} | {r * 6.0 + o for r in range(4) for o in (2.5, 3.5, 4.0, 5.5)})
    zs = [0.0, 1.0, 2.1, 2.2, H]

    def corridor_kind(i, j):
        x0 = xs[i] % 6.0
        if abs(x0 - 2.5) < 1e-9 and zs[j] < 2.1:
            return None
        if abs(x0 - 4.0) < 1e-9 and 1.0 <= zs[j] < 2.2:
            return "glass"
        return "wall"
    for y in (6.0, 8.0):
        _wall_cells(mb, 1, y, xs, zs, corridor_kind, mats)
    # partitions with a window (y in [2, 4] / [10, 12], 1.0 to 2.2 m)
    for x in (6.0, 12.0, 18.0):
        for (y0, y1) in ((0.0, 6.0), (8.0, 14.0)):
            ys = [y0, y0 + 2.0, y0 + 4.0, y1]
            _wall_cells(mb, 0, x, ys, zs, lambda i, j: "glass" if i == 1 and 1.0 <= zs[j] < 2.2 else "wall", mats)
    # receivers and transmitter off the walls' lattice, so that no path meets
    # a face edge by construction
    gx = np.arange(rx_step * 0.437, W, rx_step)
    gy = np.arange(rx_step * 0.383, D, rx_step)
    rx = np.array([[x, y, 1.5] for y in gy for x in gx], np.float32)
    tx = np.array([[3.173, 7.061, 2.0]], np.float32)
    inf = float("inf")
    return mb.finish("indoor_office", [CONCRETE, WALL_OUTDOOR, WALL_INDOOR, GLASS_INDOOR], tx, rx,
                     rx_radius=0.2, n_rays=n_rays, max_reflections=max_reflections, freqs_hz=[30e9],
                     tx_power_w=0.5, penetration_db=np.array([inf, inf, PEN_WALL_INDOOR_DB, PEN_GLASS_INDOOR_DB]),
                     max_transmissions=max_transmissions)


def box_field(n_static: int, n_moving: int, half: float = 200.0, seed: int = 5, n_frames: int = 4,
              n_rays: int = 1 << 15, max_reflections: int = 3) -> Scene:
    """Large or object-rich test scene: a ground plane with `n_static` concrete
    boxes (sides U(1, 4) m, heights U(1, 12) m) and `n_moving` metal boxes
    (2 x 1 x 1 m, 0.3 m clearance) at uniform positions in [-half, half]^2; the
    moving boxes translate at U(-15, 15) m/s per axis.  Boxes are untessellated
    (12 triangles, 6 faces each) and may overlap.  One Tx at 30 m, an 8 x 8
    receiver grid at 1.5 m.  Built with array operations so that hundreds of
    thousands of triangles stay cheap."""
    rng = np.random.default_rng(seed)
    unit = _MeshBuilder()
    unit.add_box((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (1, 1, 1), 0)
    uv, ut, uf = unit.verts[0].astype(np.float64), unit.tris[0], unit.tri_face[0]
    n_box = n_static + n_moving
    lo = np.zeros((n_box, 3))
    size = np.zeros((n_box, 3))
    lo[:, :2] = rng.uniform(-half, half, (n_box, 2))
    size[:n_static, :2] = rng.uniform(1.0, 4.0, (n_static, 2))
    size[:n_static, 2] = rng.uniform(1.0, 12.0, n_static)
    size[n_static:] = (2.0, 1.0, 1.0)
    lo[n_static:, 2] = 0.3
    verts = (lo[:, None, :] + size[:, None, :] * uv[None, :, :]).astype(np.float32)   # [n_box, 8, 3]
    nv_box = uv.shape[0]
    tris = ut[None, :, :] + (np.arange(n_box) * nv_box)[:, None, None]
    tri_face = uf[None, :] + (np.arange(n_box) * 6)[:, None]
    g = 2.0 * half + 20.0
    ground_v = np.array([[-g, -g, 0.0], [g, -g, 0.0], [g, g, 0.0], [-g, g, 0.0]], np.float32)
    nvb = n_box * nv_box
    all_v = np.concatenate([verts.reshape(-1, 3), ground_v])
    all_t = np.concatenate([tris.reshape(-1, 3), np.array([[0, 1, 2], [0, 2, 3]]) + nvb]).astype(np.int32)
    all_f = np.concatenate([tri_face.reshape(-1), [6 * n_box, 6 * n_box]]).astype(np.int32)
    face_material = np.concatenate([np.zeros(6 * n_static), np.ones(6 * n_moving), [2]]).astype(np.int32)
    face_object = np.concatenate([np.full(6 * n_static, -1), np.repeat(np.arange(n_moving), 6), [-1]]).astype(np.int32)
    obj_range = np.stack([np.arange(n_static, n_box) * nv_box, np.arange(n_static + 1, n_box + 1) * nv_box], 1)
    vel = rng.uniform(-15.0, 15.0, (n_moving, 2))
    dt = 0.1

    def transforms(frame: int) -> np.ndarray:
        xf = identity_transforms(n_moving)
        xf[:, 0, 3] = (vel[:, 0] * frame * dt).astype(np.float32)
        xf[:, 1, 3] = (vel[:, 1] * frame * dt).astype(np.float32)
        return xf

    gx = np.linspace(-0.8 * half, 0.8 * half, 8)
    rx = np.array([[x, y, 1.5] for x in gx for y in gx], np.float32)
    return Scene(name="box_field", vertices=all_v, tris=all_t, tri_face=all_f, face_material=face_material,
                 face_object=face_object, materials=np.array([CONCRETE, METAL, GROUND], np.float64),
                 object_vertex_range=obj_range.astype(np.int64), tx=np.array([[0.0, 0.0, 30.0]], np.float32),
                 rx=rx, rx_radius=0.5, n_rays=n_rays, max_reflections=max_reflections, n_frames=n_frames, dt=dt,
                 transforms_fn=transforms)


def _quad_grid(p0, p1, p3, na: int, nb: int):
    """Planar quad p0, p1, p0 + (p1 - p0) + (p3 - p0), p3 split into na x nb
    cells of two triangles: (points, triangles)."""
    p0, p1, p3 = (np.asarray(p, np.float64) for p in (p0, p1, p3))
    ea, eb = p1 - p0, p3 - p0
    pts = [p0 + ea * (i / na) + eb * (j / nb) for j in range(nb + 1) for i in range(na + 1)]
    tris = []
    for j in range(nb):
        for i in range(na):
            a = j * (na + 1) + i
            tris += [(a, a + 1, a + na + 2), (a, a + na + 2, a + na + 1)]
    return np.array(pts), tris


def _rot_z(a: float) -> np.ndarray:
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def _rot_x(a: float) -> np.ndarray:
    c, s = np.cos(a), np.sin(a)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def _box_faces(centre, half, R, cells=(1, 1, 1), skip_bottom: bool = False):
    """The six sides of the box centre + R [-half, half]^3 (R a rotation) as
    tessellated planar faces."""
    c, h = np.asarray(centre, np.float64), np.asarray(half, np.float64)

    def P(sx, sy, sz):
        return c + R @ (h * np.array([sx, sy, sz], np.float64))

    nx, ny, nz = cells
    sides = [
        (P(-1, -1, -1), P(-1, -1, 1), P(-1, 1, -1), nz, ny),   # -x
        (P(1, -1, -1), P(1, 1, -1), P(1, -1, 1), ny, nz),      # +x
        (P(-1, -1, -1), P(1, -1, -1), P(-1, -1, 1), nx, nz),   # -y
        (P(-1, 1, -1), P(-1, 1, 1), P(1, 1, -1), nz, nx),      # +y
        (P(-1, -1, -1), P(-1, 1, -1), P(1, -1, -1), ny, nx),   # -z
        (P(-1, -1, 1), P(1, -1, 1), P(-1, 1, 1), nx, ny),      # +z
    ]
    return [_quad_grid(p0, p1, p3, na, nb) for i, (p0, p1, p3, na, nb) in enumerate(sides)
            if not (skip_bottom and i == 4)]


def oblique_town(seed: int = 3, n_rays: int = 1 << 16, max_reflections: int = 3, n_frames: int = 20) -> Scene:
    """Small town whose reflecting planes are mostly oblique, with objects that
    rotate between frames.

    Ground [-150, 150]^2.  Eight concrete buildings (centres U(-100, 100)^2,
    15 m clear of the transmitter and 2 m of each other) yawed by U(0, pi/2),
    half footprints U(6, 14) m, heights U(10, 35) m, walls tessellated 2 x 3;
    half have flat roofs and half gable roofs (two slopes of U(20, 40) degrees
    with Table II's outdoor-wall coefficient 0.8, and two gable walls).  A
    static billboard 8 x 4 m tilted 35 degrees from vertical.  Moving: five
    metal cars (4.5 x 1.8 x 1.5 m boxes, 0.3 m clearance) driving round
    circles about the transmitter of radius U(20, 60) m at U(8, 16) m/s, each
    turned to its heading every frame (yaw rotations; the cars may pass
    through buildings), and a 6 x 0.3 x 2 m metal sign turning about a
    horizontal axis at 1.5 rad/s.  Transforms are relative to the frame-0
    pose.  Tx on a 12 m pole at the origin; 64 receivers uniform in
    [-100, 100]^2 outside the buildings at 1.5 m, capture radius 1 m.
    """
    rng = np.random.default_rng(seed)
    tx = np.array([[0.0, 0.0, 12.0]])
    mb = _MeshBuilder()
    mb.add_ground(150.0, material=1)
    placed = []
    n_bld = 0
    while n_bld < 8:
        hx, hy = rng.uniform(6.0, 14.0, size=2)
        h = rng.uniform(10.0, 35.0)
        yaw = rng.uniform(0.0, np.pi / 2)
        cx, cy = rng.uniform(-100.0, 100.0, size=2)
        rad = np.hypot(hx, hy)
        if np.hypot(cx, cy) < rad + 15.0:
            continue
        if any(np.hypot(cx - q[0], cy - q[1]) < rad + q[2] + 2.0 for q in placed):
            continue
        placed.append((cx, cy, rad))
        R = _rot_z(yaw)
        gable = n_bld % 2 == 1
        faces = _box_faces((cx, cy, h / 2), (hx, hy, h / 2), R, cells=(2, 2, 3), skip_bottom=True)
        if gable:
            pitch = np.radians(rng.uniform(20.0, 40.0))
            ridge = h + hy * np.tan(pitch)

            def W(lx, ly, z):
                return np.array([cx, cy, 0.0]) + R @ np.array([lx, ly, 0.0]) + np.array([0, 0, z])

            roof = [_quad_grid(W(-hx, -hy, h), W(hx, -hy, h), W(-hx, 0.0, ridge), 2, 1),
                    _quad_grid(W(-hx, hy, h), W(-hx, 0.0, ridge), W(hx, hy, h), 1, 2)]
            ends = [(np.array([W(sx, -hy, h), W(sx, hy, h), W(sx, 0.0, ridge)]), [(0, 1, 2)]) for sx in (-hx, hx)]
            mb.add_faces(faces[:4] + ends, material=0)
            mb.add_faces(roof, material=3)
        else:
            mb.add_faces(faces, material=0)
        n_bld += 1

    def inside_building(x, y, margin):
        for (cx, cy, rad) in placed:
            if np.hypot(x - cx, y - cy) < rad + margin:
                return True
        return False

    rx = []
    while len(rx) < 64:
        x, y = rng.uniform(-100.0, 100.0, size=2)
        if not inside_building(x, y, 1.0) and np.hypot(x, y) > 5.0:
            rx.append((x, y, 1.5))
    rx_all = np.array(rx)
    # tilted billboard on the side of the plaza
    Rb = _rot_z(0.6) @ _rot_x(np.radians(35.0))
    mb.add_faces([_quad_grid(*(np.array([-30.0, 25.0, 6.0]) + Rb @ np.array(p, np.float64)
                               for p in ([-4, 0, -2], [4, 0, -2], [-4, 0, 2])), 2, 1)], material=2)
    # moving objects: cars on circles (yaw), a turning sign (pitch)
    cars = []
    for v in range(5):
        r = rng.uniform(20.0, 60.0)
        th0 = rng.uniform(0.0, 2 * np.pi)
        w = rng.uniform(8.0, 16.0) / r * (1 if v % 2 == 0 else -1)
        cars.append((r, th0, w))
    dt = 0.1

    def car_pose(r, th0, w, frame):
        th = th0 + w * frame * dt
        p = np.array([r * np.cos(th), r * np.sin(th), VEHICLE_CLEARANCE + VEHICLE[2] / 2])
        return p, _rot_z(th + np.sign(w) * np.pi / 2)

    for v, (r, th0, w) in enumerate(cars):
        p, R = car_pose(r, th0, w, 0)
        mb.add_faces(_box_faces(p, np.array(VEHICLE) / 2, R), material=2, obj=v)
    sign_c = np.array([12.0, -8.0, 4.0])
    mb.add_faces(_box_faces(sign_c, (3.0, 0.15, 1.0), np.eye(3)), material=2, obj=5)

    def transforms(frame: int) -> np.ndarray:
        xf = np.zeros((6, 3, 4), np.float64)
        for v, (r, th0, w) in enumerate(cars):
            p0, R0 = car_pose(r, th0, w, 0)
            p1, R1 = car_pose(r, th0, w, frame)
            M = R1 @ R0.T                       # x' = M (x - p0) + p1
            xf[v, :, :3] = M
            xf[v, :, 3] = p1 - M @ p0
        M = _rot_x(1.5 * frame * dt)
        xf[5, :, :3] = M
        xf[5, :, 3] = sign_c - M @ sign_c
        return xf.astype(np.float32)

    return mb.finish("oblique_town", [CONCRETE, GROUND, METAL, (5.31, 0.48, 0.8)], tx, rx_all,
                     rx_radius=1.0, n_rays=n_rays, max_reflections=max_reflections, freqs_hz=[28e9],
                     tx_power_w=5.0, n_frames=n_frames, dt=dt, transforms_fn=transforms)


def _box_template(cells):
    """Unit box [0, 1]^3 tessellated into cells: (vertices, triangles, local face of each triangle)."""
    mb = _MeshBuilder()
    mb.add_box((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), cells, material=0)
    return mb.verts[0].astype(np.float64), mb.tris[0], mb.tri_face[0]


def ragged_city(seed: int, target_tris: int, n_tx: int = 1, n_rx: int = 256, n_rays: int = 1 << 18,
                max_reflections: int = 4, freqs_hz=(28e9,), n_frames: int = 10) -> Scene:
    """A grid-and-vehicles city of about `target_tris` triangles, built with
    array operations so that hundreds of thousands of triangles stay cheap.

    G x G blocks of 40 m with 15 m streets, one concrete building per block
    (height U(10, 60) m, facades tessellated t x 2t cells per side, roofs
    t x t), V metal vehicles (4.5 x 1.8 x 1.5 m, 0.3 m clearance, 512
    triangles) on random streets and lanes at U(10, 20) m/s, wrapping at the
    grid edge.  V ~ 15% of the triangle budget (2..200), then G and t fill the
    rest (G in 2..16).  n_tx transmitters on 2 m masts at roof corners of
    random blocks, n_rx receivers on sidewalks at 1.5 m (capture radius
    0.5 m).  Materials: concrete, ground, metal."""
    rng = np.random.default_rng(seed)
    V = int(np.clip(round(0.15 * target_tris / 512), 2, 200))
    rest = max(target_tris - 512 * V, 2000)
    G = int(np.clip(round(np.sqrt(rest / 2000.0)), 2, 16))
    t = max(1, int(round(np.sqrt(rest / (20.0 * G * G)))))
    extent = G * BLOCK + (G + 1) * STREET
    half = extent / 2.0
    origin = lambda i: -half + STREET + i * (BLOCK + STREET)
    centre = lambda k: -half + STREET / 2.0 + k * (BLOCK + STREET)
    heights = rng.uniform(10.0, 60.0, size=(G, G))
    bv, bt, bf = _box_template((t, t, 2 * t))
    ii, jj = np.meshgrid(np.arange(G), np.arange(G), indexing="ij")
    lo = np.stack([origin(ii.ravel()), origin(jj.ravel()), np.zeros(G * G)], 1)
    size = np.stack([np.full(G * G, BLOCK), np.full(G * G, BLOCK), heights.ravel()], 1)
    bverts = lo[:, None, :] + size[:, None, :] * bv[None]
    vv, vt, vf = _box_template((12, 5, 4))
    veh = []
    vlo, vsize = [], []
    for v in range(V):
        street = int(rng.integers(0, 2 * (G + 1)))
        lane = int(rng.integers(0, 2))
        u = rng.uniform(-half, half)
        speed = rng.uniform(10.0, 20.0)
        c = centre(street % (G + 1))
        L, W, H = VEHICLE
        if street <= G:
            axis, lane_c, dirn = 0, c - LANE_OFFSET if lane == 0 else c + LANE_OFFSET, 1.0 if lane == 0 else -1.0
            vlo.append((u - L / 2, lane_c - W / 2, VEHICLE_CLEARANCE))
            vsize.append((L, W, H))
        else:
            axis, lane_c, dirn = 1, c + LANE_OFFSET if lane == 0 else c - LANE_OFFSET, 1.0 if lane == 0 else -1.0
            vlo.append((lane_c - W / 2, u - L / 2, VEHICLE_CLEARANCE))
            vsize.append((W, L, H))
        veh.append((axis, dirn, u, speed))
    # vehicles use the template in (x, y) order; a vehicle along y swaps the cell counts' roles,
    # which only changes the tessellation pattern, not the box
    vverts = np.asarray(vlo)[:, None, :] + np.asarray(vsize)[:, None, :] * vv[None]
    n_b, n_v = G * G, V
    nbv, nvv = bv.shape[0], vv.shape[0]
    ground = np.array([[-half - 5, -half - 5, 0.0], [half + 5, -half - 5, 0.0], [half + 5, half + 5, 0.0],
                       [-half - 5, half + 5, 0.0]])
    verts = np.concatenate([ground, bverts.reshape(-1, 3), vverts.reshape(-1, 3)]).astype(np.float32)
    g_t = np.array([[0, 1, 2], [0, 2, 3]])
    b_tris = (bt[None] + 4 + (np.arange(n_b) * nbv)[:, None, None]).reshape(-1, 3)
    v_tris = (vt[None] + 4 + n_b * nbv + (np.arange(n_v) * nvv)[:, None, None]).reshape(-1, 3)
    tris = np.concatenate([g_t, b_tris, v_tris]).astype(np.int32)
    tri_face = np.concatenate([[0, 0], (bf[None] + 1 + 6 * np.arange(n_b)[:, None]).ravel(),
                               (vf[None] + 1 + 6 * n_b + 6 * np.arange(n_v)[:, None]).ravel()]).astype(np.int32)
    face_material = np.concatenate([[1], np.zeros(6 * n_b), np.full(6 * n_v, 2)]).astype(np.int32)
    face_object = np.concatenate([[-1], np.full(6 * n_b, -1), np.repeat(np.arange(n_v), 6)]).astype(np.int32)
    v0 = 4 + n_b * nbv
    obj_range = np.stack([v0 + np.arange(n_v) * nvv, v0 + (np.arange(n_v) + 1) * nvv], 1).astype(np.int64)
    # transmitters: 2 m masts 0.5 m inside a roof corner of random blocks
    txs = []
    for k in range(n_tx):
        i, j = rng.integers(0, G, size=2)
        txs.append((origin(i) + BLOCK - 0.5, origin(j) + BLOCK - 0.5, heights[i, j] + 2.0))
    centres = np.array([centre(k) for k in range(G + 1)])
    rx = []
    while len(rx) < n_rx:
        street = int(rng.integers(0, 2 * (G + 1)))
        side = 1.0 if rng.integers(0, 2) == 1 else -1.0
        off = rng.uniform(4.5, 7.0)
        along = rng.uniform(-half + 2.5, half - 2.5)
        if np.any(np.abs(along - centres) < STREET / 2 + 0.5):
            continue
        c = centres[street % (G + 1)]
        rx.append((along, c + side * off, 1.5) if street <= G else (c + side * off, along, 1.5))
    dt = 0.1

    def transforms(frame: int) -> np.ndarray:
        xf = identity_transforms(n_v)
        for v, (axis, dirn, u, speed) in enumerate(veh):
            p_ = u + dirn * speed * frame * dt
            p_ = -half + np.mod(p_ + half, extent)
            xf[v, axis, 3] = np.float32(p_ - u)
        return xf

    return Scene(name="ragged_city", vertices=verts, tris=tris, tri_face=tri_face, face_material=face_material,
                 face_object=face_object, materials=np.array([CONCRETE, GROUND, METAL], np.float64),
                 object_vertex_range=obj_range, tx=np.array(txs, np.float32), rx=np.array(rx, np.float32),
                 rx_radius=0.5, n_rays=n_rays, max_reflections=max_reflections, freqs_hz=list(freqs_hz),
                 n_frames=n_frames, dt=dt, transforms_fn=transforms)


def highway_city(seed: int = 5, grid_blocks: int = 16, facade_cells: int = 19, corridor_m: float = 6000.0,
                 warehouses: int = 60, n_vehicles: int = 200, n_rx: int = 4096, n_tx: int = 4,
                 n_rays: int = 1 << 22, max_reflections: int = 6, freqs_hz=(28e9, 60e9),
                 n_frames: int = 300) -> Scene:
    """Large dynamic scene: a highway corridor beside a city grid, with
    receivers mounted on the moving vehicles.

    City: grid_blocks^2 blocks of 40 m with 15 m streets centred on the
    origin, concrete buildings of height U(10, 60) m, facades tessellated
    facade_cells x 2 facade_cells per side.  Corridor: a straight highway of
    corridor_m along x, 60 m south of the grid, four lanes (centres +-2 and
    +-6 m), 4 m concrete noise barriers 12 m either side of the centre line
    (4 m x 2 m cells), and `warehouses` 50 x 25 m buildings (height U(8, 16) m)
    behind each barrier.  n_vehicles metal vehicles (4.5 x 1.8 x 1.5 m, 512
    triangles), 60% on the highway lanes and 40% on the city streets, at
    U(15, 35) m/s, wrapping at the ends.  n_rx receivers on the vehicle roofs
    (0.2 m above, spread over each roof), moving with them.  n_tx roadside
    transmitters on 10 m poles 9 m north of the centre line, evenly along the
    corridor.  With the defaults about 2M triangles."""
    rng = np.random.default_rng(seed)
    G = grid_blocks
    extent = G * BLOCK + (G + 1) * STREET
    half = extent / 2.0
    origin = lambda i: -half + STREET + i * (BLOCK + STREET)
    centre = lambda k: -half + STREET / 2.0 + k * (BLOCK + STREET)
    yc = -(half + 60.0)   # corridor centre line
    Lc = corridor_m
    parts_v, parts_t, parts_f, mats, objs = [], [], [], [], []
    nv = 0
    nfaces = 0

    def add_boxes(lo, size, cells, material, obj_ids=None):
        nonlocal nv, nfaces
        tv, tt, tf = _box_template(cells)
        n = lo.shape[0]
        verts = lo[:, None, :] + size[:, None, :] * tv[None]
        parts_v.append(verts.reshape(-1, 3))
        parts_t.append((tt[None] + nv + (np.arange(n) * tv.shape[0])[:, None, None]).reshape(-1, 3))
        parts_f.append((tf[None] + nfaces + 6 * np.arange(n)[:, None]).ravel())
        mats.append(np.full(6 * n, material))
        objs.append(np.full(6 * n, -1) if obj_ids is None else np.repeat(obj_ids, 6))
        first = nv
        nv += n * tv.shape[0]
        nfaces += 6 * n
        return first, tv.shape[0]

    # ground (one face)
    x0, x1 = -Lc / 2 - 50.0, Lc / 2 + 50.0
    y0, y1 = yc - 100.0, half + 20.0
    parts_v.append(np.array([[x0, y0, 0.0], [x1, y0, 0.0], [x1, y1, 0.0], [x0, y1, 0.0]]))
    parts_t.append(np.array([[0, 1, 2], [0, 2, 3]]))
    parts_f.append(np.array([0, 0]))
    mats.append(np.array([1]))
    objs.append(np.array([-1]))
    nv, nfaces = 4, 1
    # city buildings
    heights = rng.uniform(10.0, 60.0, size=(G, G))
    ii, jj = np.meshgrid(np.arange(G), np.arange(G), indexing="ij")
    lo = np.stack([origin(ii.ravel()), origin(jj.ravel()), np.zeros(G * G)], 1)
    size = np.stack([np.full(G * G, BLOCK), np.full(G * G, BLOCK), heights.ravel()], 1)
    add_boxes(lo, size, (facade_cells, facade_cells, 2 * facade_cells), 0)
    # noise barriers: thin boxes 0.3 m thick, 4 m tall
    n_seg = max(1, int(round(Lc / 200.0)))
    seg_len = Lc / n_seg
    bx = -Lc / 2 + seg_len * np.arange(n_seg)
    for side in (-1.0, 1.0):
        lo = np.stack([bx, np.full(n_seg, yc + side * 12.0 - 0.15), np.zeros(n_seg)], 1)
        size = np.stack([np.full(n_seg, seg_len), np.full(n_seg, 0.3), np.full(n_seg, 4.0)], 1)
        add_boxes(lo, size, (int(seg_len / 4.0), 1, 2), 0)
    # warehouses behind the barriers
    if warehouses > 0:
        wx = -Lc / 2 + (np.arange(warehouses) + 0.5) * (Lc / warehouses) - 25.0
        for side in (-1.0, 1.0):
            y_lo = yc + side * 25.0 - (25.0 if side < 0 else 0.0)
            lo = np.stack([wx, np.full(warehouses, y_lo), np.zeros(warehouses)], 1)
            size = np.stack([np.full(warehouses, 50.0), np.full(warehouses, 25.0), rng.uniform(8.0, 16.0, warehouses)], 1)
            add_boxes(lo, size, (10, 5, 4), 0)
    # vehicles
    L, W, H = VEHICLE
    veh = []   # (axis, dir, u, speed, lo_xyz, size_xyz, lane period start, period)
    n_hw = int(round(0.6 * n_vehicles))
    lanes = [(-6.0, -1.0), (-2.0, -1.0), (2.0, 1.0), (6.0, 1.0)]
    v_lo, v_size = [], []
    for v in range(n_vehicles):
        speed = rng.uniform(15.0, 35.0)
        if v < n_hw:
            off, dirn = lanes[int(rng.integers(0, 4))]
            u = rng.uniform(-Lc / 2, Lc / 2)
            veh.append((0, dirn, u, speed, -Lc / 2, Lc))
            v_lo.append((u - L / 2, yc + off - W / 2, VEHICLE_CLEARANCE))
            v_size.append((L, W, H))
        else:
            street = int(rng.integers(0, 2 * (G + 1)))
            lane = int(rng.integers(0, 2))
            u = rng.uniform(-half, half)
            c = centre(street % (G + 1))
            if street <= G:
                lane_c, dirn = (c - LANE_OFFSET, 1.0) if lane == 0 else (c + LANE_OFFSET, -1.0)
                veh.append((0, dirn, u, speed, -half, extent))
                v_lo.append((u - L / 2, lane_c - W / 2, VEHICLE_CLEARANCE))
                v_size.append((L, W, H))
            else:
                lane_c, dirn = (c + LANE_OFFSET, 1.0) if lane == 0 else (c - LANE_OFFSET, -1.0)
                veh.append((1, dirn, u, speed, -half, extent))
                v_lo.append((lane_c - W / 2, u - L / 2, VEHICLE_CLEARANCE))
                v_size.append((W, L, H))
    v_lo, v_size = np.asarray(v_lo), np.asarray(v_size)
    v_first, v_nv = add_boxes(v_lo, v_size, (12, 5, 4), 2, obj_ids=np.arange(n_vehicles))
    verts = np.concatenate(parts_v).astype(np.float32)
    tris = np.concatenate(parts_t).astype(np.int32)
    tri_face = np.concatenate(parts_f).astype(np.int32)
    face_material = np.concatenate(mats).astype(np.int32)
    face_object = np.concatenate(objs).astype(np.int32)
    obj_range = np.stack([v_first + np.arange(n_vehicles) * v_nv, v_first + (np.arange(n_vehicles) + 1) * v_nv],
                         1).astype(np.int64)
    # receivers on the roofs: vehicle of each receiver and its roof position
    rv = np.arange(n_rx) % n_vehicles
    slot = np.arange(n_rx) // n_vehicles
    per = np.bincount(rv, minlength=n_vehicles)
    rx0 = np.zeros((n_rx, 3))
    for r in range(n_rx):
        v, k, m = rv[r], slot[r], max(per[rv[r]], 1)
        f = (k + 0.5) / m
        rx0[r] = (v_lo[v, 0] + v_size[v, 0] * (0.1 + 0.8 * f if veh[v][0] == 0 else 0.5),
                  v_lo[v, 1] + v_size[v, 1] * (0.1 + 0.8 * f if veh[v][0] == 1 else 0.5),
                  VEHICLE_CLEARANCE + H + 0.2)
    txs = [(-Lc / 2 + (k + 0.5) * Lc / n_tx, yc + 9.0, 10.0) for k in range(n_tx)]
    dt = 0.1

    def shifts(frame: int) -> np.ndarray:
        out = np.zeros((n_vehicles, 3))
        for v, (axis, dirn, u, speed, start, period) in enumerate(veh):
            p_ = u + dirn * speed * frame * dt
            p_ = start + np.mod(p_ - start, period)
            out[v, axis] = np.float32(p_ - u)
        return out

    def transforms(frame: int) -> np.ndarray:
        xf = identity_transforms(n_vehicles)
        xf[:, :, 3] = shifts(frame).astype(np.float32)
        return xf

    def rx_fn(frame: int) -> np.ndarray:
        return (rx0 + shifts(frame)[rv]).astype(np.float32)

    return Scene(name="highway_city", vertices=verts, tris=tris, tri_face=tri_face, face_material=face_material,
                 face_object=face_object, materials=np.array([CONCRETE, GROUND, METAL], np.float64),
                 object_vertex_range=obj_range, tx=np.array(txs, np.float32), rx=rx_fn(0), rx_radius=0.5,
                 n_rays=n_rays, max_reflections=max_reflections, freqs_hz=list(freqs_hz), n_frames=n_frames,
                 dt=dt, transforms_fn=transforms, rx_fn=rx_fn)


def batched_workload(n_scenes: int = 64, seed: int = 3, tri_range=(10_000, 500_000), budget_range=(1 << 18, 1 << 22),
                     rx_range=(64, 1024), tx_range=(1, 8), k_range=(2, 6), bands=(28e9, 60e9)):
    """Ragged batch of independent cities: triangle counts and ray budgets
    log-uniform over their ranges, 1-8 transmitters (the budget is split
    over them), 2-6 reflections, 64-1024 receivers and one band (28 or 60 GHz)
    per scene, all from `seed`."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_scenes):
        tris = int(np.exp(rng.uniform(np.log(tri_range[0]), np.log(tri_range[1]))))
        budget = int(np.exp(rng.uniform(np.log(budget_range[0]), np.log(budget_range[1]))))
        n_tx = int(rng.integers(tx_range[0], tx_range[1] + 1))
        n_rx = int(np.exp(rng.uniform(np.log(rx_range[0]), np.log(rx_range[1]))))
        K = int(rng.integers(k_range[0], k_range[1] + 1))
        band = float(bands[int(rng.integers(0, len(bands)))])
        out.append(ragged_city(seed * 1000 + k, tris, n_tx=n_tx, n_rx=n_rx, n_rays=max(budget // n_tx, 1),
                               max_reflections=K, freqs_hz=(band,)))
    return out


def random_sphere_dirs(n: int, seed: int) -> np.ndarray:
    """n random directions, uniform on the unit sphere (the paper's 'random sphere of rays')."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v.astype(np.float32)


CONFIGS = {
    "static_toy": static_toy,
    "dynamic_urban": dynamic_urban,
    "oblique_town": oblique_town,
}
