"""FP64 CPU oracle of the explicit MPM step -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps the plain C implementation in
``mpm_oracle.c`` (built with gcc, no FMA contraction) and shares no code with
the GPU library.

Scene descriptions are plain dicts with the keys produced by the seeded input
generators: ``mesh`` {n, origin, h}, ``material`` {model, rho, E, nu, phi,
psi, c, dp_cone}, ``bc`` {face, extra, force}, ``scheme`` {algo, shape, gravity, dt,
mass_eps_rel, velocity_update}, and particle arrays x (n,3), v (n,3),
stress (n,6), vol (n,), mass (n,), all float64.

What each C function follows is stated in ``mpm_oracle.h``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mpm_oracle.c")
_LIBPATH = os.path.join(_HERE, "libmpm_oracle.so")

LINEAR_ELASTIC, DRUCKER_PRAGER = 0, 1
DP_OUTER, DP_INNER, DP_PLANE_STRAIN = 0, 1, 2
FREE, FIXED, SLIP = 0, 1, 2
USF, USL, MUSL = 0, 1, 2
SHAPE_LINEAR, SHAPE_GIMP = 0, 1
FLIP, PIC = 0, 1

OK, E_ARG, E_NOMEM, E_OUT_OF_MESH, E_NONFINITE = 0, -1, -2, -4, -5


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle error {code}")
        self.code = code


def build() -> str:
    """Compile the oracle shared library (gcc, -O2, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-Wall", "-fPIC",
           "-shared", "-o", _LIBPATH + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIBPATH + ".tmp", _LIBPATH)
    return _LIBPATH


class _Mesh(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("pad_", ctypes.c_int32),
                ("origin", ctypes.c_double * 3), ("h", ctypes.c_double),
                ("node_x", ctypes.POINTER(ctypes.c_double))]


class _Material(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("dp_cone", ctypes.c_int32),
                ("rho", ctypes.c_double), ("E", ctypes.c_double), ("nu", ctypes.c_double),
                ("phi", ctypes.c_double), ("psi", ctypes.c_double), ("c", ctypes.c_double)]


class _Bc(ctypes.Structure):
    _fields_ = [("face", ctypes.c_int32 * 6), ("pad_", ctypes.c_int32),
                ("n_extra", ctypes.c_int64),
                ("node", ctypes.POINTER(ctypes.c_int64)),
                ("axis", ctypes.POINTER(ctypes.c_int32)),
                ("value", ctypes.POINTER(ctypes.c_double)),
                ("n_force", ctypes.c_int64),
                ("force_node", ctypes.POINTER(ctypes.c_int64)),
                ("force_value", ctypes.POINTER(ctypes.c_double)),
                ("force_ramp_steps", ctypes.c_int64)]


class _Scheme(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("shape", ctypes.c_int32),
                ("velocity_update", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("gravity", ctypes.c_double * 3), ("dt", ctypes.c_double),
                ("mass_eps_rel", ctypes.c_double)]


class _Grid(ctypes.Structure):
    _fields_ = [("m", ctypes.POINTER(ctypes.c_double)), ("p", ctypes.POINTER(ctypes.c_double)),
                ("v", ctypes.POINTER(ctypes.c_double)), ("f", ctypes.POINTER(ctypes.c_double)),
                ("a", ctypes.POINTER(ctypes.c_double)), ("vn", ctypes.POINTER(ctypes.c_double)),
                ("cell_count", ctypes.POINTER(ctypes.c_uint32))]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH) or os.path.getmtime(_LIBPATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIBPATH)
    P = ctypes.POINTER
    d, i32, i64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64
    lib.om_num_nodes.argtypes = [P(_Mesh), i32]
    lib.om_num_nodes.restype = i64
    lib.om_num_cells.argtypes = [P(_Mesh)]
    lib.om_num_cells.restype = i64
    lib.om_node_id.argtypes = [P(_Mesh), i32, i64, i64, i64]
    lib.om_node_id.restype = i64
    lib.om_locate.argtypes = [P(_Mesh), i64, P(d), P(i64)]
    lib.om_locate.restype = ctypes.c_int
    lib.om_shape.argtypes = [P(_Mesh), i32, P(d), P(i64), P(d), P(d)]
    lib.om_shape.restype = ctypes.c_int
    lib.om_iso_natural.argtypes = [P(_Mesh), P(i64), P(d), P(d)]
    lib.om_iso_natural.restype = ctypes.c_int
    lib.om_gimp_1d.argtypes = [d, d, d, P(d)]
    lib.om_gimp_1d.restype = None
    lib.om_dp_coefficients.argtypes = [P(_Material), P(d)]
    lib.om_dp_coefficients.restype = None
    lib.om_constitutive.argtypes = [P(_Material), P(d), P(d)]
    lib.om_constitutive.restype = ctypes.c_int
    step_args = [P(_Mesh), P(_Material), P(_Bc), P(_Scheme), i64, P(d), P(d), P(d), P(d), P(d), P(_Grid), i64]
    lib.om_step.argtypes = step_args
    lib.om_step.restype = ctypes.c_int
    lib.om_run.argtypes = step_args + [i64]
    lib.om_run.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a, ctype=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _mesh(mesh: dict) -> _Mesh:
    """The C mesh descriptor; an isoparametric mesh (``node_x``, (nodes, 3)
    float64) is referenced, and kept alive by the descriptor."""
    m = _Mesh()
    for a in range(3):
        m.n[a] = int(mesh["n"][a])
        m.origin[a] = float(mesh["origin"][a])
    m.h = float(mesh["h"])
    if mesh.get("node_x") is not None:
        nx = np.ascontiguousarray(mesh["node_x"], dtype=np.float64).reshape(-1, 3)
        want = (m.n[0] + 1) * (m.n[1] + 1) * (m.n[2] + 1)
        if len(nx) != want:
            raise ValueError(f"node_x holds {len(nx)} nodes, the mesh has {want}")
        m._keep = nx
        m.node_x = _ptr(nx)
    return m


def _material(mat: dict) -> _Material:
    return _Material(int(mat["model"]), int(mat.get("dp_cone", DP_OUTER)), float(mat["rho"]),
                     float(mat["E"]), float(mat["nu"]), float(mat.get("phi", 0.0)),
                     float(mat.get("psi", 0.0)), float(mat.get("c", 0.0)))


def _scheme(sch: dict) -> _Scheme:
    s = _Scheme()
    s.algo = int(sch.get("algo", USF))
    s.shape = int(sch.get("shape", SHAPE_LINEAR))
    s.velocity_update = int(sch.get("velocity_update", FLIP))
    for a in range(3):
        s.gravity[a] = float(sch["gravity"][a])
    s.dt = float(sch["dt"])
    s.mass_eps_rel = float(sch.get("mass_eps_rel", 1e-10))
    return s


class _BcHolder:
    """Keeps the arrays behind an om_bc alive for the duration of a call."""

    def __init__(self, bc: dict):
        self.c = _Bc()
        for k in range(6):
            self.c.face[k] = int(bc["face"][k])
        extra = bc.get("extra")
        if extra is not None and len(extra[0]) > 0:
            self.node = np.ascontiguousarray(extra[0], dtype=np.int64)
            self.axis = np.ascontiguousarray(extra[1], dtype=np.int32)
            self.value = np.ascontiguousarray(extra[2], dtype=np.float64)
            self.c.n_extra = len(self.node)
            self.c.node = _ptr(self.node, ctypes.c_int64)
            self.c.axis = _ptr(self.axis, ctypes.c_int32)
            self.c.value = _ptr(self.value)
        else:
            self.c.n_extra = 0
        force = bc.get("force")
        if force is not None and len(force[0]) > 0:
            self.fnode = np.ascontiguousarray(force[0], dtype=np.int64)
            self.fval = np.ascontiguousarray(np.asarray(force[1], dtype=np.float64).reshape(len(self.fnode), 3))
            self.c.n_force = len(self.fnode)
            self.c.force_node = _ptr(self.fnode, ctypes.c_int64)
            self.c.force_value = _ptr(self.fval)
            self.c.force_ramp_steps = int(bc.get("force_ramp_steps", 0))
        else:
            self.c.n_force = 0


def num_nodes(mesh: dict, shape: int = SHAPE_LINEAR) -> int:
    return int(_load().om_num_nodes(ctypes.byref(_mesh(mesh)), shape))


def num_cells(mesh: dict) -> int:
    return int(_load().om_num_cells(ctypes.byref(_mesh(mesh))))


def node_id(mesh: dict, shape: int, i: int, j: int, k: int) -> int:
    return int(_load().om_node_id(ctypes.byref(_mesh(mesh)), shape, i, j, k))


def locate(mesh: dict, x: np.ndarray) -> np.ndarray:
    """Linear cell id of each particle (raises OracleError if outside)."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    cell = np.empty(len(x), dtype=np.int64)
    rc = _load().om_locate(ctypes.byref(_mesh(mesh)), len(x), _ptr(x), _ptr(cell, ctypes.c_int64))
    if rc != OK:
        raise OracleError(rc, "locate")
    return cell


def cell_counts(mesh: dict, x: np.ndarray) -> np.ndarray:
    """Particles per cell in linear cell order (uint32)."""
    cell = locate(mesh, x)
    return np.bincount(cell, minlength=num_cells(mesh)).astype(np.uint32)


def shape(mesh: dict, shape_kind: int, xp) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(node ids, N, dN/dx) of one particle's support."""
    xp = np.ascontiguousarray(xp, dtype=np.float64)
    node = np.empty(27, dtype=np.int64)
    N = np.empty(27)
    dN = np.empty(81)
    q = _load().om_shape(ctypes.byref(_mesh(mesh)), shape_kind, _ptr(xp), _ptr(node, ctypes.c_int64),
                         _ptr(N), _ptr(dN))
    if q < 0:
        raise OracleError(q, "shape")
    return node[:q].copy(), N[:q].copy(), dN[:3 * q].reshape(q, 3).copy()


def iso_natural(mesh: dict, cell, x) -> tuple[np.ndarray, int]:
    """Natural coordinates of x in cell (cx, cy, cz) of an isoparametric
    mesh and the Newton iterations taken (raises OracleError on breakdown)."""
    c = np.ascontiguousarray(cell, dtype=np.int64)
    xp = np.ascontiguousarray(x, dtype=np.float64)
    xi = np.empty(3)
    it = _load().om_iso_natural(ctypes.byref(_mesh(mesh)), _ptr(c, ctypes.c_int64), _ptr(xp), _ptr(xi))
    if it < 0:
        raise OracleError(it, "iso_natural")
    return xi, int(it)


def gimp_1d(r: float, h: float, l: float) -> tuple[float, float]:
    out = np.empty(2)
    _load().om_gimp_1d(float(r), float(h), float(l), _ptr(out))
    return float(out[0]), float(out[1])


def dp_coefficients(mat: dict) -> tuple[float, float, float]:
    out = np.empty(3)
    _load().om_dp_coefficients(ctypes.byref(_material(mat)), _ptr(out))
    return float(out[0]), float(out[1]), float(out[2])


def constitutive(mat: dict, deps, sig) -> tuple[np.ndarray, int]:
    """One stress update; returns (new stress, 0 elastic / 1 cone / 2 apex)."""
    deps = np.ascontiguousarray(deps, dtype=np.float64)
    s = np.array(sig, dtype=np.float64)
    kind = _load().om_constitutive(ctypes.byref(_material(mat)), _ptr(deps), _ptr(s))
    return s, int(kind)


class Grid:
    """Caller-owned nodal workspace; after a step holds that step's fields."""

    def __init__(self, mesh: dict, shape_kind: int):
        nn = num_nodes(mesh, shape_kind)
        self.m = np.zeros(nn)
        self.p = np.zeros((nn, 3))
        self.v = np.zeros((nn, 3))
        self.f = np.zeros((nn, 3))
        self.a = np.zeros((nn, 3))
        self.vn = np.zeros((nn, 3))
        self.cell_count = np.zeros(num_cells(mesh), dtype=np.uint32)
        self.c = _Grid(_ptr(self.m), _ptr(self.p), _ptr(self.v), _ptr(self.f), _ptr(self.a),
                       _ptr(self.vn), _ptr(self.cell_count, ctypes.c_uint32))


def run(scene: dict, nsteps: int, grid: Grid | None = None, state: dict | None = None) -> dict:
    """Advance a scene by nsteps; returns the particle state (x, v, stress,
    vol, mass), the count of steps done since the scene's start
    (``steps_done``) and the grid of the last step.  ``state`` (if given,
    e.g. an earlier return value) replaces the scene's initial particle
    arrays and continues its step count."""
    src = state if state is not None else scene
    step0 = int(state.get("steps_done", 0)) if state is not None else 0
    x = np.array(src["x"], dtype=np.float64, order="C").reshape(-1, 3)
    v = np.array(src["v"], dtype=np.float64, order="C").reshape(-1, 3)
    n = len(x)
    sig = np.array(src["stress"], dtype=np.float64, order="C").reshape(n, 6) if src.get("stress") is not None \
        else np.zeros((n, 6))
    vol = np.array(src["vol"], dtype=np.float64, order="C").reshape(n)
    mass = np.array(src["mass"], dtype=np.float64, order="C").reshape(n)
    sch = _scheme(scene["scheme"])
    if grid is None:
        grid = Grid(scene["mesh"], sch.shape)
    bch = _BcHolder(scene["bc"])
    rc = _load().om_run(ctypes.byref(_mesh(scene["mesh"])), ctypes.byref(_material(scene["material"])),
                        ctypes.byref(bch.c), ctypes.byref(sch), n, _ptr(x), _ptr(v), _ptr(sig),
                        _ptr(vol), _ptr(mass), ctypes.byref(grid.c), step0, int(nsteps))
    if rc != OK:
        raise OracleError(rc, "run")
    return {"x": x, "v": v, "stress": sig, "vol": vol, "mass": mass, "grid": grid,
            "steps_done": step0 + int(nsteps)}
