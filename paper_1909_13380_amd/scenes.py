"""Seeded synthetic scene inputs for the explicit MPM step.

This module only *generates inputs* (mesh, particle positions, velocities,
volumes, masses, material constants, boundary rules, time step); it holds
none of the method's arithmetic and imports nothing from the GPU library or
the oracle, so both can be fed the same arrays.

A scene is a plain dict:
  mesh     {"n": (nx, ny, nz), "origin": (ox, oy, oz), "h": h}
  material {"model", "dp_cone", "rho", "E", "nu", "phi", "psi", "c"}  (angles in radians)
  bc       {"face": [-x, +x, -y, +y, -z, +z] rules, "extra": None or (node ids, axes, values),
            "force": absent, None or (node ids, forces (k, 3))}
  scheme   {"algo", "shape", "velocity_update", "gravity", "dt", "mass_eps_rel"}
  x (n,3) float64; v (n,3), vol (n,), mass (n,), stress (n,6) float64 holding
  float32-representable values (so an FP32 consumer starts from exactly the
  same numbers); nsteps; name.

Particle layouts: "gauss" puts 2x2x2 particles per cell at the natural
coordinates +-1/sqrt(3) (offsets h(1 -+ 1/sqrt3)/2); "centre" puts them at the
sub-cell centres (h/4, 3h/4) plus an optional uniform jitter of +-10% of the
particle spacing h/2.  Particle volume is h^3/8 and mass rho*volume.
"""
from __future__ import annotations

import math

import numpy as np

LINEAR_ELASTIC, DRUCKER_PRAGER = 0, 1
DP_OUTER, DP_INNER, DP_PLANE_STRAIN = 0, 1, 2
FREE, FIXED, SLIP = 0, 1, 2
USF, USL, MUSL = 0, 1, 2
SHAPE_LINEAR, SHAPE_GIMP = 0, 1
FLIP, PIC = 0, 1

GRAVITY = (0.0, 0.0, -9.81)
SOIL = {"rho": 1800.0, "E": 10.0e6, "nu": 0.3}


def _f32(a) -> np.ndarray:
    """Round to float32 and hold as float64 (exactly representable in both)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def elastic(rho=SOIL["rho"], E=SOIL["E"], nu=SOIL["nu"]) -> dict:
    return {"model": LINEAR_ELASTIC, "dp_cone": DP_OUTER, "rho": rho, "E": E, "nu": nu,
            "phi": 0.0, "psi": 0.0, "c": 0.0}


def drucker_prager(phi_deg=30.0, psi_deg=0.0, c=0.0, cone=DP_OUTER, rho=SOIL["rho"], E=SOIL["E"],
                   nu=SOIL["nu"]) -> dict:
    return {"model": DRUCKER_PRAGER, "dp_cone": cone, "rho": rho, "E": E, "nu": nu,
            "phi": math.radians(phi_deg), "psi": math.radians(psi_deg), "c": c}


def p_wave_speed(mat: dict) -> float:
    """Dilatational wave speed sqrt((K + 4G/3)/rho), used to pick dt by CFL."""
    E, nu, rho = mat["E"], mat["nu"], mat["rho"]
    M = E * (1.0 - nu) / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return math.sqrt(M / rho)


def block_positions(lo, hi, h, origin=(0.0, 0.0, 0.0), layout="centre", jitter=0.0, rng=None) -> np.ndarray:
    """Particle positions filling cells lo[a] <= c < hi[a], 2x2x2 per cell.

    Order: cells in x-fastest order, the 8 particles of a cell in x-fastest
    order.  jitter is a fraction of the particle spacing h/2.
    """
    lo = np.asarray(lo, dtype=np.int64)
    hi = np.asarray(hi, dtype=np.int64)
    if layout == "gauss":
        off = np.array([0.5 * (1.0 - 1.0 / math.sqrt(3.0)), 0.5 * (1.0 + 1.0 / math.sqrt(3.0))])
    else:
        off = np.array([0.25, 0.75])
    cz, cy, cx = np.meshgrid(np.arange(lo[2], hi[2]), np.arange(lo[1], hi[1]), np.arange(lo[0], hi[0]),
                             indexing="ij")
    cells = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1).astype(np.float64)
    kz, ky, kx = np.meshgrid(off, off, off, indexing="ij")
    sub = np.stack([kx.ravel(), ky.ravel(), kz.ravel()], axis=1)
    x = (cells[:, None, :] + sub[None, :, :]).reshape(-1, 3) * h + np.asarray(origin, dtype=np.float64)
    if jitter:
        rng = rng if rng is not None else np.random.default_rng(0)
        x = x + rng.uniform(-jitter * 0.5 * h, jitter * 0.5 * h, size=x.shape)
    return x


def make_scene(name, mesh, material, bc, scheme, x, v=None, nsteps=1, stress=None) -> dict:
    n = len(x)
    h = mesh["h"]
    vol = _f32(np.full(n, h ** 3 / 8.0))
    mass = _f32(material["rho"] * vol)
    v = _f32(np.zeros((n, 3)) if v is None else v)
    stress = _f32(np.zeros((n, 6)) if stress is None else stress)
    return {"name": name, "mesh": mesh, "material": material, "bc": bc, "scheme": scheme,
            "x": np.ascontiguousarray(x, dtype=np.float64), "v": v, "vol": vol, "mass": mass,
            "stress": stress, "nsteps": int(nsteps)}


def scheme(dt, shape=SHAPE_LINEAR, algo=USF, gravity=GRAVITY, velocity_update=FLIP, mass_eps_rel=1e-10) -> dict:
    return {"algo": algo, "shape": shape, "velocity_update": velocity_update, "gravity": tuple(gravity),
            "dt": float(dt), "mass_eps_rel": mass_eps_rel}


def walls(floor=SLIP, sides=SLIP, top=FREE) -> dict:
    return {"face": [sides, sides, sides, sides, floor, top], "extra": None}


# --------------------------------------------------------------- configs --

def c1(seed: int = 1) -> dict:
    """Elastic block of 8x8x8 cells on the floor at the centre of a 16^3 mesh
    (h = 0.1 m), 2x2x2 Gauss-position particles per cell (4,096 particles),
    velocities uniform in +-0.01 m/s, gravity, fixed floor, roller walls,
    dt = 1e-4 s, 200 steps."""
    h = 0.1
    mesh = {"n": (16, 16, 16), "origin": (0.0, 0.0, 0.0), "h": h}
    x = block_positions((4, 4, 0), (12, 12, 8), h, layout="gauss")
    rng = np.random.default_rng(seed)
    v = rng.uniform(-0.01, 0.01, size=x.shape)
    return make_scene("c1", mesh, elastic(), walls(floor=FIXED, sides=SLIP), scheme(1e-4), x, v, nsteps=200)


def c2(seed: int = 2) -> dict:
    """Granular column collapse: Drucker-Prager block of 64x32x128 cells
    against the x = 0 wall, centred in y, on a 256x128x160 mesh (h = 0.01 m),
    8 particles per cell jittered +-10% of spacing (2,097,152 particles),
    frictionless walls, dt = 2e-5 s, 1000 steps."""
    h = 0.01
    mesh = {"n": (256, 128, 160), "origin": (0.0, 0.0, 0.0), "h": h}
    rng = np.random.default_rng(seed)
    x = block_positions((0, 48, 0), (64, 80, 128), h, layout="centre", jitter=0.1, rng=rng)
    return make_scene("c2", mesh, drucker_prager(), walls(), scheme(2e-5), x, None, nsteps=1000)


def column(cells, mesh_cells, h, dt, seed, nsteps, shape=SHAPE_LINEAR, name="column") -> dict:
    """A Drucker-Prager column of `cells` against x = 0, centred in y, on the
    floor of a `mesh_cells` mesh: the C2/C5 recipe at any size."""
    bx, by, bz = cells
    ny = mesh_cells[1]
    y0 = (ny - by) // 2
    mesh = {"n": tuple(int(c) for c in mesh_cells), "origin": (0.0, 0.0, 0.0), "h": h}
    rng = np.random.default_rng(seed)
    x = block_positions((0, y0, 0), (bx, y0 + by, bz), h, layout="centre", jitter=0.1, rng=rng)
    return make_scene(name, mesh, drucker_prager(), walls(), scheme(dt, shape=shape), x, None, nsteps=nsteps)


def c5(seed: int = 5, subsample: bool = False, shape: int = SHAPE_GIMP) -> dict:
    """Drucker-Prager block of 256x128x96 cells on a 512x256x128 mesh of
    0.005 m cells, GIMP, 25,165,824 particles, dt = 1e-5 s, 500 steps.  The
    1/64 subsample divides every extent by 4 (64x32x24 block on 128x64x32)."""
    if subsample:
        return column((64, 32, 24), (128, 64, 32), 0.005, 1e-5, seed, 500, shape, "c5_sub")
    return column((256, 128, 96), (512, 256, 128), 0.005, 1e-5, seed, 500, shape, "c5")


PLATE = {"h": 0.0625, "radius": 0.5, "half_length": 4.0, "half_width": 2.5, "sigma0": 100.0}


def plate_end_forces(mesh: dict, sigma0: float, end_i: int, width_cells: int) -> tuple:
    """Nodal forces equivalent to a uniform traction sigma0 (along +x) on the
    strip's end face x = end_i h, which spans width_cells cells in y and the
    mesh's one cell in z: each bilinear face element of h x h carries
    sigma0 h^2 / 4 to each of its four corner nodes.  Node ids in the
    library's numbering (linear shape functions)."""
    h = mesh["h"]
    n0, n1 = mesh["n"][0] + 1, mesh["n"][1] + 1
    f = {}
    for j in range(width_cells):
        for k in range(mesh["n"][2]):
            for dj in (0, 1):
                for dk in (0, 1):
                    node = end_i + n0 * ((j + dj) + n1 * (k + dk))
                    f[node] = f.get(node, 0.0) + sigma0 * h * h / 4.0
    ids = sorted(f)
    return ids, np.array([[f[i], 0.0, 0.0] for i in ids])


def plate_with_hole(load: str = "traction", load_time: float = 1.0, hold_time: float = 0.0,
                    points_per_axis: int = 4, material=None) -> dict:
    """The paper's validation strip (benchmark section, Table 1): 5 m wide,
    8 m long, a centred hole of radius 0.5 m, in uniaxial tension of 100 Pa
    along its length (x), cells of 0.0625 m.  The quarter x, y >= 0 is
    modelled with symmetry (slip) faces at x = 0 and y = 0, as one layer of
    cells with 4 x 4 points per cell (all at mid-thickness) and a slip face
    at z = 0 and a free one at z = h, which leaves sigma_zz free (plane
    stress).  Points are the sub-cell centres outside the hole: 40,153 of
    them (the paper has 40,156).

    load="traction" (the paper's load): sigma0 = 100 Pa on the end face
    x = 4 m as nodal forces (plate_end_forces), ramped linearly from zero
    over `load_time` seconds and then held for `hold_time`.  load="pulled":
    the end's nodes move along x at the constant velocity that reaches the
    nominal strain sigma0 / E at `load_time` (per-node velocity
    constraints).  The mesh leaves two empty cell columns beyond the end.
    PIC velocity update (it damps the motion), no gravity, explicit USF,
    linear shape functions, dt at a CFL number of 0.3."""
    P = PLATE
    h, a, L, W = P["h"], P["radius"], P["half_length"], P["half_width"]
    nx, ny = int(round(L / h)), int(round(W / h))
    mesh = {"n": (nx + 2, ny + 1, 1), "origin": (0.0, 0.0, 0.0), "h": h}
    g = (np.arange(nx * points_per_axis) + 0.5) * (h / points_per_axis)
    q = (np.arange(ny * points_per_axis) + 0.5) * (h / points_per_axis)
    X, Y = np.meshgrid(g, q, indexing="ij")
    keep = X * X + Y * Y >= a * a
    x = np.stack([X[keep], Y[keep], np.full(int(keep.sum()), h / 2)], axis=1)
    mat = material or elastic()
    dt = 0.3 * h / p_wave_speed(mat)
    nsteps = int(round(load_time / dt))
    if load == "traction":
        bc = {"face": [SLIP, FREE, SLIP, FREE, SLIP, FREE], "extra": None,
              "force": plate_end_forces(mesh, P["sigma0"], nx, ny), "force_ramp_steps": nsteps}
        nsteps += int(round(hold_time / dt))
    elif load == "pulled":
        speed = P["sigma0"] / mat["E"] * L / load_time
        n0, n1 = mesh["n"][0] + 1, mesh["n"][1] + 1
        ids = [nx + n0 * (j + n1 * k) for k in range(2) for j in range(n1)]
        bc = {"face": [SLIP, FREE, SLIP, FREE, SLIP, FREE], "extra": (ids, [0] * len(ids), [speed] * len(ids))}
    else:
        raise ValueError(f"unknown plate load {load!r}")
    sc = make_scene("plate_with_hole", mesh, mat, bc,
                    scheme(dt, gravity=(0.0, 0.0, 0.0), velocity_update=PIC), x, None, nsteps=nsteps)
    sc["vol"] = _f32(np.full(len(x), h ** 3 / points_per_axis ** 2))
    sc["mass"] = _f32(mat["rho"] * sc["vol"])
    return sc


def c3_scene(index: int, h: float = 0.02, nsteps: int = 500) -> dict:
    """Scene `index` of the batched set: particle count log-uniform in
    [1e3, 2.5e5] (8 per cell), horizontal aspect ratios log-uniform in
    [0.5, 2], mesh = block padded 50% on each horizontal side and 1.5x the
    block height (+1 cell), elastic (even seed) or Drucker-Prager (odd seed),
    dt from a CFL number of 0.3 on the dilatational wave speed."""
    seed = 3000 + index
    rng = np.random.default_rng(seed)
    P = math.exp(rng.uniform(math.log(1e3), math.log(2.5e5)))
    C = P / 8.0
    ax = math.exp(rng.uniform(math.log(0.5), math.log(2.0)))
    ay = math.exp(rng.uniform(math.log(0.5), math.log(2.0)))
    nz = max(2, int(round((C / (ax * ay)) ** (1.0 / 3.0))))
    nx = max(2, int(round(ax * nz)))
    ny = max(2, int(round(ay * nz)))
    mesh_n = (2 * nx, 2 * ny, int(math.ceil(1.5 * nz)) + 1)
    mesh = {"n": mesh_n, "origin": (0.0, 0.0, 0.0), "h": h}
    x0, y0 = (mesh_n[0] - nx) // 2, (mesh_n[1] - ny) // 2
    x = block_positions((x0, y0, 0), (x0 + nx, y0 + ny, nz), h, layout="centre", jitter=0.1, rng=rng)
    if seed % 2 == 0:
        mat, bc = elastic(), walls(floor=FIXED, sides=SLIP)
    else:
        mat, bc = drucker_prager(), walls()
    dt = 0.3 * h / p_wave_speed(mat)
    return make_scene(f"c3_{index}", mesh, mat, bc, scheme(dt), x, None, nsteps=nsteps)


def c3(n_scenes: int = 256, nsteps: int = 500) -> list:
    return [c3_scene(i, nsteps=nsteps) for i in range(n_scenes)]


def c4_requests(rate_hz: float, n_requests: int, seed: int = 4, scene_offset: int = 4000) -> list:
    """Poisson request stream drawn from the batched-scene generator: each
    request is (arrival time in s, scene, step count uniform in 100..2000)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n_requests))
    steps = rng.integers(100, 2001, size=n_requests)
    out = []
    for i in range(n_requests):
        sc = c3_scene(scene_offset - 3000 + i, nsteps=int(steps[i]))
        out.append((float(t[i]), sc, int(steps[i])))
    return out


def column_requests(rate_hz: float, n_requests: int, seed: int = 4, scene_offset: int = 5000) -> list:
    """Poisson request stream drawn from the granular column generator (C2's
    2,097,152-particle Drucker-Prager column): each request is (arrival time
    in s, scene, step count uniform in 100..2000), every scene with its own
    jitter seed (scene_offset + request index).  The scenes share every
    array but the positions."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n_requests))
    steps = rng.integers(100, 2001, size=n_requests)
    base = c2()
    h = base["mesh"]["h"]
    centres = block_positions((0, 48, 0), (64, 80, 128), h, layout="centre")
    out = []
    for i in range(n_requests):
        jr = np.random.default_rng(scene_offset + i)
        x = centres + jr.uniform(-0.1 * 0.5 * h, 0.1 * 0.5 * h, size=centres.shape)
        sc = dict(base, x=x, name=f"column_{i}", nsteps=int(steps[i]))
        out.append((float(t[i]), sc, int(steps[i])))
    return out


# ------------------------------------------------ closed-form test scenes --

def free_body(v0=(0.3, -0.2, 0.1), gravity=GRAVITY, cells=(4, 3, 5), mesh_cells=(16, 16, 16), h=0.1,
              dt=1e-4, shape=SHAPE_LINEAR, material=None, nsteps=50) -> dict:
    """A body with uniform velocity v0 well away from every wall, all faces
    free: free fall under gravity (or rigid translation with gravity 0)."""
    lo = tuple((m - c) // 2 for m, c in zip(mesh_cells, cells))
    hi = tuple(l + c for l, c in zip(lo, cells))
    mesh = {"n": tuple(mesh_cells), "origin": (0.0, 0.0, 0.0), "h": h}
    x = block_positions(lo, hi, h, layout="centre")
    v = np.tile(np.asarray(v0, dtype=np.float64), (len(x), 1))
    return make_scene("free_body", mesh, material or elastic(), walls(floor=FREE, sides=FREE),
                      scheme(dt, shape=shape, gravity=gravity), x, v, nsteps=nsteps)


def elastic_bar(n_cells=20, h=0.05, v0=1e-3, cfl=0.1, rho=1800.0, E=10.0e6, shape=SHAPE_LINEAR) -> dict:
    """Fixed-free bar along x (nu = 0), one cell of cross-section between
    roller walls, 2x2x2 Gauss particles per cell, first-mode velocity
    v0 sin(pi x / 2L), no gravity.  dt = cfl * h / sqrt(E/rho)."""
    L = n_cells * h
    mesh = {"n": (n_cells + 2, 1, 1), "origin": (0.0, 0.0, 0.0), "h": h}
    x = block_positions((0, 0, 0), (n_cells, 1, 1), h, layout="gauss")
    v = np.zeros_like(x)
    v[:, 0] = v0 * np.sin(np.pi * x[:, 0] / (2.0 * L))
    c = math.sqrt(E / rho)
    bc = {"face": [FIXED, FREE, SLIP, SLIP, SLIP, SLIP], "extra": None}
    return make_scene("elastic_bar", mesh, elastic(rho=rho, E=E, nu=0.0), bc,
                      scheme(cfl * h / c, shape=shape, gravity=(0.0, 0.0, 0.0)), x, v, nsteps=0)


def random_block(n_cells=(6, 5, 4), mesh_cells=(12, 10, 8), h=0.05, seed=11, material=None, bc=None,
                 shape=SHAPE_LINEAR, dt=2e-5, vel=0.5, gravity=GRAVITY, stress_scale=0.0, nsteps=5,
                 jitter=0.4) -> dict:
    """Small irregular test scene: a jittered block with random velocities
    (and optionally random initial stress) resting on the floor, centred."""
    rng = np.random.default_rng(seed)
    lo = ((mesh_cells[0] - n_cells[0]) // 2, (mesh_cells[1] - n_cells[1]) // 2, 0)
    hi = tuple(l + c for l, c in zip(lo, n_cells))
    mesh = {"n": tuple(mesh_cells), "origin": (0.0, 0.0, 0.0), "h": h}
    x = block_positions(lo, hi, h, layout="centre", jitter=jitter, rng=rng)
    v = rng.uniform(-vel, vel, size=x.shape)
    stress = rng.uniform(-stress_scale, stress_scale, size=(len(x), 6)) if stress_scale else None
    return make_scene("random_block", mesh, material or elastic(), bc or walls(floor=FIXED),
                      scheme(dt, shape=shape, gravity=gravity), x, v, nsteps=nsteps, stress=stress)


# ------------------------------------------------ isoparametric meshes --

def _smooth_field(mesh: dict, amp: float, seed: int):
    """A smooth displacement field d(X) of amplitude amp * h over the mesh's
    box: component a is amp h sin(pi m_a (X_a - o_a) / L_a) times cosines
    of the other two coordinates with random phases, so it vanishes on the
    two faces normal to axis a (those faces stay planar).  Returns d and its
    gradient as functions of positions (k, 3)."""
    rng = np.random.default_rng(seed)
    h = mesh["h"]
    o = np.asarray(mesh["origin"], dtype=np.float64)
    L = np.asarray(mesh["n"], dtype=np.float64) * h
    m = rng.integers(1, 3, size=3)
    ph = rng.uniform(0, 2 * np.pi, size=(3, 3))
    A = amp * h * rng.uniform(0.5, 1.0, size=3)

    def parts(X):
        u = (np.asarray(X, dtype=np.float64) - o) / L          # in [0, 1] over the box
        out = np.zeros_like(u)
        grad = np.zeros(u.shape + (3,))
        for a in range(3):
            b, c = (a + 1) % 3, (a + 2) % 3
            s = np.sin(np.pi * m[a] * u[:, a])
            cb = np.cos(2 * np.pi * u[:, b] + ph[a, b])
            cc = np.cos(2 * np.pi * u[:, c] + ph[a, c])
            out[:, a] = A[a] * s * cb * cc
            grad[:, a, a] = A[a] * np.pi * m[a] / L[a] * np.cos(np.pi * m[a] * u[:, a]) * cb * cc
            grad[:, a, b] = -A[a] * 2 * np.pi / L[b] * s * np.sin(2 * np.pi * u[:, b] + ph[a, b]) * cc
            grad[:, a, c] = -A[a] * 2 * np.pi / L[c] * s * cb * np.sin(2 * np.pi * u[:, c] + ph[a, c])
        return out, grad
    return parts


def uniform_nodes(mesh: dict) -> np.ndarray:
    """Node positions o + h (i, j, k) of a mesh in node-id order (n+1 per axis)."""
    n = mesh["n"]
    k, j, i = np.meshgrid(np.arange(n[2] + 1), np.arange(n[1] + 1), np.arange(n[0] + 1), indexing="ij")
    ijk = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64)
    return np.asarray(mesh["origin"], dtype=np.float64) + mesh["h"] * ijk


def distort(scene: dict, amp: float = 0.25, seed: int = 0) -> dict:
    """The same scene on an isoparametric mesh: the mesh's nodes and the
    particles are moved by one smooth displacement field of amplitude amp * h
    (_smooth_field), each particle's volume and mass scaled by the field's
    volume change det(I + grad d) at its reference position.  The mesh keeps
    origin and h (the undistorted grid it came from) beside node_x."""
    sc = dict(scene)
    mesh = dict(scene["mesh"])
    field = _smooth_field(mesh, amp, seed)
    X = uniform_nodes(mesh)
    dX, _ = field(X)
    mesh["node_x"] = X + dX
    sc["mesh"] = mesh
    dx, grad = field(scene["x"])
    sc["x"] = scene["x"] + dx
    J = np.linalg.det(np.eye(3)[None] + grad)
    sc["vol"] = _f32(scene["vol"] * J)
    sc["mass"] = _f32(scene["mass"] * J)
    return sc


def rotate(scene: dict, R, b=(0.0, 0.0, 0.0)) -> dict:
    """The scene moved rigidly by x -> R x + b: an isoparametric mesh whose
    nodes are the moved nodes, and moved particles, velocities, stresses and
    gravity (walls keep their rules on the moved faces, so use it with free
    faces)."""
    R = np.asarray(R, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    sc = dict(scene)
    mesh = dict(scene["mesh"])
    X = scene["mesh"].get("node_x")
    X = uniform_nodes(mesh) if X is None else np.asarray(X)
    mesh["node_x"] = X @ R.T + b
    sc["mesh"] = mesh
    sc["x"] = scene["x"] @ R.T + b
    sc["v"] = scene["v"] @ R.T
    S = scene["stress"]
    T = np.zeros((len(S), 3, 3))
    for (a, c), k in {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (1, 2): 4, (0, 2): 5}.items():
        T[:, a, c] = T[:, c, a] = S[:, k]
    T = R[None] @ T @ R.T[None]
    sc["stress"] = np.stack([T[:, 0, 0], T[:, 1, 1], T[:, 2, 2], T[:, 0, 1], T[:, 1, 2], T[:, 0, 2]], axis=1)
    sch = dict(scene["scheme"])
    sch["gravity"] = tuple(R @ np.asarray(scene["scheme"]["gravity"], dtype=np.float64))
    sc["scheme"] = sch
    return sc


def slope(cells=(24, 8, 10), block=(10, 8, 6), h=0.02, angle_deg=20.0, dt=None, seed=9, material=None,
          nsteps=200) -> dict:
    """A granular block on an inclined bed (the non-prismatic boundary an
    isoparametric mesh follows): a terrain-following mesh whose node (i,j,k)
    sits at (i h, j h, z_b(i h) + k h) with the bed z_b(x) = x tan(angle),
    a fixed (no-slip) bed, slip side walls in y, free ends in x and top.  The
    Drucker-Prager block fills `block` cells at the upslope end (largest x),
    2x2x2 particles per cell at the sub-cell centres, jittered."""
    mesh = {"n": tuple(int(c) for c in cells), "origin": (0.0, 0.0, 0.0), "h": h}
    t = np.tan(np.radians(angle_deg))
    X = uniform_nodes(mesh)
    X[:, 2] += X[:, 0] * t
    mesh["node_x"] = X
    rng = np.random.default_rng(seed)
    ref = block_positions((cells[0] - block[0], 0, 0), (cells[0], block[1], block[2]), h, layout="centre",
                          jitter=0.1, rng=rng)
    x = ref.copy()
    x[:, 2] += x[:, 0] * t            # sheared with the mesh (volume-preserving)
    mat = material or drucker_prager()
    dt = dt or 0.3 * h / p_wave_speed(mat)
    bc = {"face": [FREE, FREE, SLIP, SLIP, FIXED, FREE], "extra": None}
    return make_scene("slope", mesh, mat, bc, scheme(dt), x, None, nsteps=nsteps)
