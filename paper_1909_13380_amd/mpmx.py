"""ctypes binding of libmpmx (C ABI in include/mpmx.h): argument marshalling
only -- every step of the method runs in the library's HIP kernels.

Importing this module loads ``libmpmx.so`` from this package directory and
raises ImportError if it has not been built (``python -m
paper_1909_13380_amd.build``); there is no fallback implementation.

Scenes are described by the dicts of ``paper_1909_13380_amd.scenes``.
Particle arrays may be numpy arrays (host) or torch CUDA float64 tensors
(device); torch is used only for device memory and streams.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libmpmx.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "mpmx.h")

if not os.path.exists(LIBPATH):
    raise ImportError(f"{LIBPATH} is not built; run `python -m paper_1909_13380_amd.build`")
# torch ships its own HIP runtime under the same soname as the system one.
# Loading torch first makes the library bind to that runtime, so one runtime
# serves the whole process and torch streams and device pointers are valid
# here; loading the library first would leave torch a second runtime that
# finds no GPU.
try:
    import torch  # noqa: F401
except ImportError:   # no torch: the system HIP runtime is used
    torch = None
_lib = ctypes.CDLL(LIBPATH)

OK = 0
E_INVALID_ARG, E_OOM, E_BUDGET, E_OUT_OF_MESH, E_NONFINITE, E_HIP, E_AGAIN, E_NOT_FOUND, E_STATE = \
    -1, -2, -3, -4, -5, -6, -7, -8, -9
LINEAR_ELASTIC, DRUCKER_PRAGER = 0, 1
USF, USL, MUSL = 0, 1, 2
SHAPE_LINEAR, SHAPE_GIMP = 0, 1
FLIP, PIC = 0, 1
FP32, FP64 = 0, 1
SORT_ON_DEMAND, SORT_ALWAYS = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1
ERRBIT_OUT_OF_MESH, ERRBIT_NONFINITE, ERRBIT_TILE, ERRBIT_SORT = 1, 2, 4, 8
OPT_GRAPH_STEPS, OPT_AUTOTUNE, OPT_STRESS_THREADS, OPT_G2P_THREADS, OPT_BLOCKS_PER_CU, OPT_GRAPH_LAUNCHES, \
    OPT_TUNE_RUNS, OPT_STRESS_BLOCKS_PER_CU, OPT_G2P_BLOCKS_PER_CU = 1, 2, 3, 4, 5, 6, 7, 8, 9
TUNE_MIN_STEPS = 40

_P = ctypes.POINTER
_d, _i32, _i64, _u32, _u64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64


class MpmxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mpmx error {code}: {msg}")
        self.code = code


class Mesh(ctypes.Structure):
    _fields_ = [("size", _u32), ("n", _i32 * 3), ("origin", _d * 3), ("h", _d), ("node_x", _P(_d))]


class Material(ctypes.Structure):
    _fields_ = [("size", _u32), ("model", _i32), ("dp_cone", _i32), ("pad_", _i32), ("rho", _d), ("E", _d),
                ("nu", _d), ("phi", _d), ("psi", _d), ("c", _d)]


class Bc(ctypes.Structure):
    _fields_ = [("size", _u32), ("face", _i32 * 6), ("n_extra", _i64), ("node", _P(_i64)), ("axis", _P(_i32)),
                ("value", _P(_d)), ("n_force", _i64), ("force_node", _P(_i64)), ("force_value", _P(_d)),
                ("force_ramp_steps", _i64)]


class Scheme(ctypes.Structure):
    _fields_ = [("size", _u32), ("algo", _i32), ("shape", _i32), ("velocity_update", _i32), ("precision", _i32),
                ("sort_policy", _i32), ("gravity", _d * 3), ("dt", _d), ("mass_eps_rel", _d)]


class Particles(ctypes.Structure):
    _fields_ = [("size", _u32), ("mem", _i32), ("n", _i64), ("x", ctypes.c_void_p), ("v", ctypes.c_void_p),
                ("stress", ctypes.c_void_p), ("vol", ctypes.c_void_p), ("mass", ctypes.c_void_p)]


class ParticlesOut(ctypes.Structure):
    _fields_ = [("size", _u32), ("mem", _i32), ("x", ctypes.c_void_p), ("v", ctypes.c_void_p),
                ("stress", ctypes.c_void_p), ("vol", ctypes.c_void_p), ("cell", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("size", _u32), ("n_particles", _i64), ("steps_done", _i64), ("n_sorts", _i64), ("n_items", _i64),
                ("active_cells", _i64), ("error_bits", _u32), ("pad_", _u32), ("device_bytes", _u64),
                ("pic_hash", _u64), ("lost_particles", _i64)]


class Request(ctypes.Structure):
    _fields_ = [("size", _u32), ("flags", _u32), ("mesh", _P(Mesh)), ("material", _P(Material)), ("bc", _P(Bc)),
                ("scheme", _P(Scheme)), ("particles", _P(Particles)), ("nsteps", _i64), ("tag", _u64),
                ("out", _P(ParticlesOut))]


REQ_BORROW = 1


class Completion(ctypes.Structure):
    _fields_ = [("size", _u32), ("status", _i32), ("request", _u64), ("tag", _u64), ("n", _i64),
                ("steps_done", _i64), ("x", _P(_d)), ("v", _P(_d)), ("stress", _P(_d)), ("vol", _P(_d)),
                ("t_submit", _d), ("t_admit", _d), ("t_done", _d)]


_vp = ctypes.c_void_p
_SIGNATURES = {
    "mpmx_version": ([], ctypes.c_int),
    "mpmx_create": ([_P(_vp), ctypes.c_int, _vp], ctypes.c_int),
    "mpmx_destroy": ([_vp], None),
    "mpmx_last_error": ([_vp], ctypes.c_char_p),
    "mpmx_set_option": ([_vp, ctypes.c_int, _i64], ctypes.c_int),
    "mpmx_get_option": ([_vp, ctypes.c_int, _P(_i64)], ctypes.c_int),
    "mpmx_profile_enable": ([_vp, ctypes.c_int], ctypes.c_int),
    "mpmx_profile_reset": ([_vp], ctypes.c_int),
    "mpmx_profile_read": ([_vp, ctypes.c_int, _P(ctypes.c_char_p), _P(_i64), _P(_d), _P(ctypes.c_int)],
                          ctypes.c_int),
    "mpmx_scene_bytes": ([_P(Mesh), _P(Scheme), _i64, _P(_u64)], ctypes.c_int),
    "mpmx_scene_create": ([_vp, _P(Mesh), _P(Material), _P(Bc), _P(Scheme), _P(Particles), _P(_u64)],
                          ctypes.c_int),
    "mpmx_scene_step": ([_vp, _u64, _i64], ctypes.c_int),
    "mpmx_scene_read": ([_vp, _u64, _P(ParticlesOut)], ctypes.c_int),
    "mpmx_scene_cell_counts": ([_vp, _u64, _vp, _i32], ctypes.c_int),
    "mpmx_scene_nodes": ([_vp, _u64, _vp, _vp, _vp], ctypes.c_int),
    "mpmx_scene_stats": ([_vp, _u64, _P(Stats)], ctypes.c_int),
    "mpmx_scene_destroy": ([_vp, _u64], ctypes.c_int),
    "mpmx_batch_step": ([_vp, _P(_u64), _P(_i64), ctypes.c_int], ctypes.c_int),
    "mpmx_batch_step_noalloc": ([_vp, _P(_u64), _P(_i64), ctypes.c_int], ctypes.c_int),
    "mpmx_server_create": ([_vp, _u64, _i64, _P(_vp)], ctypes.c_int),
    "mpmx_server_submit": ([_vp, _P(Request), _P(_u64)], ctypes.c_int),
    "mpmx_server_tick": ([_vp, _P(ctypes.c_int), _P(ctypes.c_int)], ctypes.c_int),
    "mpmx_server_poll": ([_vp, _P(Completion), ctypes.c_int, _P(ctypes.c_int)], ctypes.c_int),
    "mpmx_server_release": ([_vp, _u64], ctypes.c_int),
    "mpmx_server_clock": ([_vp], _d),
    "mpmx_server_set_fill": ([_vp, _i64], ctypes.c_int),
    "mpmx_fence_record": ([_vp, _P(_u64)], ctypes.c_int),
    "mpmx_fence_wait": ([_vp, _u64, ctypes.c_int, _P(ctypes.c_int)], ctypes.c_int),
    "mpmx_fence_release": ([_vp, _u64], ctypes.c_int),
    "mpmx_server_destroy": ([_vp], None),
}
for _name, (_args, _res) in _SIGNATURES.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def declared_functions(header: str = HEADER) -> list[str]:
    """Names of the functions declared in include/mpmx.h."""
    text = open(header).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(mpmx_\w+)\s*\(", text, flags=re.M)))


def version() -> int:
    return _lib.mpmx_version()


def _mesh(m: dict) -> Mesh:
    """The C mesh descriptor; an isoparametric mesh's node positions
    (``node_x``, (nodes, 3)) are referenced and kept alive by it."""
    out = Mesh()
    out.size = ctypes.sizeof(Mesh)
    for a in range(3):
        out.n[a] = int(m["n"][a])
        out.origin[a] = float(m["origin"][a])
    out.h = float(m["h"])
    if m.get("node_x") is not None:
        nx = np.ascontiguousarray(m["node_x"], dtype=np.float64).reshape(-1, 3)
        out._keep = nx
        out.node_x = nx.ctypes.data_as(_P(_d))
    return out


def _material(m: dict) -> Material:
    return Material(ctypes.sizeof(Material), int(m["model"]), int(m.get("dp_cone", 0)), 0, float(m["rho"]),
                    float(m["E"]), float(m["nu"]), float(m.get("phi", 0.0)), float(m.get("psi", 0.0)),
                    float(m.get("c", 0.0)))


def _scheme(s: dict, precision: int, sort_policy: int) -> Scheme:
    out = Scheme()
    out.size = ctypes.sizeof(Scheme)
    out.algo = int(s.get("algo", USF))
    out.shape = int(s.get("shape", SHAPE_LINEAR))
    out.velocity_update = int(s.get("velocity_update", FLIP))
    out.precision = int(precision)
    out.sort_policy = int(sort_policy)
    for a in range(3):
        out.gravity[a] = float(s["gravity"][a])
    out.dt = float(s["dt"])
    out.mass_eps_rel = float(s.get("mass_eps_rel", 1e-10))
    return out


def scene_bytes(scene: dict, precision: int = FP32, n_particles: int | None = None) -> int:
    out = _u64()
    n = len(scene["x"]) if n_particles is None else int(n_particles)
    rc = _lib.mpmx_scene_bytes(ctypes.byref(_mesh(scene["mesh"])),
                               ctypes.byref(_scheme(scene["scheme"], precision, SORT_ON_DEMAND)), n,
                               ctypes.byref(out))
    if rc != OK:
        raise MpmxError(rc, "scene_bytes")
    return int(out.value)


def _bc(bc: dict, keep: list) -> Bc:
    cbc = Bc()
    cbc.size = ctypes.sizeof(Bc)
    for k in range(6):
        cbc.face[k] = int(bc["face"][k])
    extra = bc.get("extra")
    if extra is not None and len(extra[0]) > 0:
        node = np.ascontiguousarray(extra[0], dtype=np.int64)
        axis = np.ascontiguousarray(extra[1], dtype=np.int32)
        value = np.ascontiguousarray(extra[2], dtype=np.float64)
        keep += [node, axis, value]
        cbc.n_extra = len(node)
        cbc.node = node.ctypes.data_as(_P(_i64))
        cbc.axis = axis.ctypes.data_as(_P(_i32))
        cbc.value = value.ctypes.data_as(_P(_d))
    force = bc.get("force")
    if force is not None and len(force[0]) > 0:
        fnode = np.ascontiguousarray(force[0], dtype=np.int64)
        fval = np.ascontiguousarray(np.asarray(force[1], dtype=np.float64).reshape(len(fnode), 3))
        keep += [fnode, fval]
        cbc.n_force = len(fnode)
        cbc.force_node = fnode.ctypes.data_as(_P(_i64))
        cbc.force_value = fval.ctypes.data_as(_P(_d))
        cbc.force_ramp_steps = int(bc.get("force_ramp_steps", 0))
    return cbc


def _host_f64(a, shape):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shape))


def _is_torch_cuda(a) -> bool:
    return type(a).__module__.startswith("torch") and getattr(a, "is_cuda", False)


class Context:
    """A library context on one GPU; `stream` is a raw hipStream_t handle
    (e.g. ``torch.cuda.current_stream().cuda_stream``) or None."""

    def __init__(self, device: int = 0, stream: int | None = None):
        self._h = _vp()
        rc = _lib.mpmx_create(ctypes.byref(self._h), int(device), _vp(stream) if stream else None)
        if rc != OK:
            raise MpmxError(rc, f"cannot create a context on HIP device {device}")
        self.scenes: dict[int, Scene] = {}

    def _check(self, rc: int, what: str):
        if rc != OK:
            msg = _lib.mpmx_last_error(self._h)
            raise MpmxError(rc, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if self._h:
            _lib.mpmx_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- scenes
    def create_scene(self, scene: dict, precision: int = FP32, sort_policy: int = SORT_ON_DEMAND,
                     state: dict | None = None) -> "Scene":
        """Upload a scene (dict from ``scenes``); ``state`` may replace the
        particle arrays (numpy, or torch CUDA float64 tensors)."""
        src = state if state is not None else scene
        keep = []
        cbc = _bc(scene["bc"], keep)
        parts = Particles()
        parts.size = ctypes.sizeof(Particles)
        x = src["x"]
        if _is_torch_cuda(x):
            fields = [src["x"], src["v"], src.get("stress"), src["vol"], src["mass"]]
            for t in fields:
                if t is not None and (not _is_torch_cuda(t) or str(t.dtype) != "torch.float64"
                                      or not t.is_contiguous()):
                    raise MpmxError(E_INVALID_ARG, "device inputs must be contiguous CUDA float64 tensors")
            parts.mem = MEM_DEVICE
            parts.n = int(x.shape[0])
            ptrs = [t.data_ptr() if t is not None else None for t in fields]
            keep += fields
        else:
            n = len(x)
            arrs = [_host_f64(src["x"], (n, 3)), _host_f64(src["v"], (n, 3)),
                    _host_f64(src["stress"], (n, 6)) if src.get("stress") is not None else None,
                    _host_f64(src["vol"], (n,)), _host_f64(src["mass"], (n,))]
            keep += arrs
            parts.mem = MEM_HOST
            parts.n = n
            ptrs = [a.ctypes.data if a is not None else None for a in arrs]
        parts.x, parts.v, parts.stress, parts.vol, parts.mass = ptrs
        sid = _u64()
        rc = _lib.mpmx_scene_create(self._h, ctypes.byref(_mesh(scene["mesh"])),
                                    ctypes.byref(_material(scene["material"])), ctypes.byref(cbc),
                                    ctypes.byref(_scheme(scene["scheme"], precision, sort_policy)),
                                    ctypes.byref(parts), ctypes.byref(sid))
        self._check(rc, "scene_create")
        s = Scene(self, int(sid.value), scene, precision, int(parts.n))
        self.scenes[s.id] = s
        return s

    def batch_step(self, scenes: list, nsteps):
        n = len(scenes)
        ids = (_u64 * n)(*[s.id for s in scenes])
        if np.isscalar(nsteps):
            nsteps = [int(nsteps)] * n
        ns = (_i64 * n)(*[int(k) for k in nsteps])
        self._check(_lib.mpmx_batch_step(self._h, ids, ns, n), "batch_step")

    def fence(self) -> int:
        """mpmx_fence_record: a fence after the steps queued so far."""
        f = _u64()
        self._check(_lib.mpmx_fence_record(self._h, ctypes.byref(f)), "fence_record")
        return int(f.value)

    def fence_done(self, fence: int, block: bool = False) -> bool:
        """mpmx_fence_wait: True once the fence's work has finished (the fence
        is then freed); with block, waits for it."""
        d = ctypes.c_int(0)
        self._check(_lib.mpmx_fence_wait(self._h, int(fence), 1 if block else 0, ctypes.byref(d)), "fence_wait")
        return bool(d.value)

    def batch_step_noalloc(self, scenes: list, nsteps):
        """mpmx_batch_step_noalloc: the same steps, with no device allocation."""
        n = len(scenes)
        ids = (_u64 * n)(*[s.id for s in scenes])
        if np.isscalar(nsteps):
            nsteps = [int(nsteps)] * n
        ns = (_i64 * n)(*[int(k) for k in nsteps])
        self._check(_lib.mpmx_batch_step_noalloc(self._h, ids, ns, n), "batch_step_noalloc")

    # -- profiling
    def set_option(self, option: int, value: int):
        self._check(_lib.mpmx_set_option(self._h, int(option), int(value)), "set_option")

    def get_option(self, option: int) -> int:
        v = _i64()
        self._check(_lib.mpmx_get_option(self._h, int(option), ctypes.byref(v)), "get_option")
        return int(v.value)

    def profile(self, enable: bool = True):
        self._check(_lib.mpmx_profile_enable(self._h, 1 if enable else 0), "profile_enable")

    def profile_reset(self):
        self._check(_lib.mpmx_profile_reset(self._h), "profile_reset")

    def profile_read(self) -> dict:
        """{kernel name: (launches, total ms)} from HIP events."""
        n = ctypes.c_int()
        self._check(_lib.mpmx_profile_read(self._h, 0, None, None, None, ctypes.byref(n)), "profile_read")
        cap = n.value
        names = (ctypes.c_char_p * max(cap, 1))()
        launches = (_i64 * max(cap, 1))()
        ms = (_d * max(cap, 1))()
        self._check(_lib.mpmx_profile_read(self._h, cap, names, launches, ms, ctypes.byref(n)), "profile_read")
        return {names[i].decode(): (int(launches[i]), float(ms[i])) for i in range(min(cap, n.value))}


class Scene:
    def __init__(self, ctx: Context, sid: int, desc: dict, precision: int, n: int):
        self.ctx, self.id, self.desc, self.precision, self.n = ctx, sid, desc, precision, n

    def step(self, nsteps: int = 1):
        self.ctx._check(_lib.mpmx_scene_step(self.ctx._h, self.id, int(nsteps)), "scene_step")

    def read(self, device_out: dict | None = None, raise_on_error: bool = True) -> dict:
        """Particle state in input order as numpy arrays (or into the given
        torch CUDA float64 tensors): x, v, stress, vol, cell."""
        out = ParticlesOut()
        out.size = ctypes.sizeof(ParticlesOut)
        n = self.n
        if device_out is not None:
            out.mem = MEM_DEVICE
            res = device_out
            for k in ("x", "v", "stress", "vol", "cell"):
                t = device_out.get(k)
                setattr(out, k, t.data_ptr() if t is not None else None)
        else:
            out.mem = MEM_HOST
            res = {"x": np.empty((n, 3)), "v": np.empty((n, 3)), "stress": np.empty((n, 6)),
                   "vol": np.empty(n), "cell": np.empty(n, dtype=np.int32)}
            for k, a in res.items():
                setattr(out, k, a.ctypes.data)
        rc = _lib.mpmx_scene_read(self.ctx._h, self.id, ctypes.byref(out))
        if rc != OK and (raise_on_error or rc not in (E_OUT_OF_MESH, E_NONFINITE)):
            self.ctx._check(rc, "scene_read")
        return res

    def cell_counts(self) -> np.ndarray:
        nc = int(np.prod(self.desc["mesh"]["n"]))
        out = np.empty(nc, dtype=np.uint32)
        self.ctx._check(_lib.mpmx_scene_cell_counts(self.ctx._h, self.id, out.ctypes.data, MEM_HOST),
                        "scene_cell_counts")
        return out

    def num_nodes(self) -> int:
        g = 1 if self.desc["scheme"].get("shape", 0) == SHAPE_GIMP else 0
        return int(np.prod([c + 1 + 2 * g for c in self.desc["mesh"]["n"]]))

    def nodes(self) -> dict:
        nn = self.num_nodes()
        m, p, f = np.empty(nn), np.empty((nn, 3)), np.empty((nn, 3))
        self.ctx._check(_lib.mpmx_scene_nodes(self.ctx._h, self.id, m.ctypes.data, p.ctypes.data, f.ctypes.data),
                        "scene_nodes")
        return {"m": m, "p": p, "f": f}

    def stats(self) -> dict:
        st = Stats()
        st.size = ctypes.sizeof(Stats)
        self.ctx._check(_lib.mpmx_scene_stats(self.ctx._h, self.id, ctypes.byref(st)), "scene_stats")
        return {k: int(getattr(st, k)) for k, _ in Stats._fields_ if k not in ("size", "pad_")}

    def destroy(self):
        if self.id:
            self.ctx._check(_lib.mpmx_scene_destroy(self.ctx._h, self.id), "scene_destroy")
            self.ctx.scenes.pop(self.id, None)
            self.id = 0


class Server:
    """Request loop over a context (mpmx_server_*): submit scenes at any
    time, call tick() to admit and advance them, poll() for finished ones."""

    def __init__(self, ctx: Context, budget_bytes: int, max_tick_steps: int = 256, fill_particles: int = 0):
        self.ctx = ctx
        self._h = _vp()
        rc = _lib.mpmx_server_create(ctx._h, int(budget_bytes), int(max_tick_steps), ctypes.byref(self._h))
        if rc != OK:
            raise MpmxError(rc, "server_create")
        self._held = {}   # request id -> (borrowed inputs, output arrays) until polled
        if fill_particles:
            self.set_fill(fill_particles)

    def set_fill(self, particles: int):
        """Admission waits while scenes still stepping hold >= particles (0: off)."""
        rc = _lib.mpmx_server_set_fill(self._h, int(particles))
        if rc != OK:
            raise MpmxError(rc, "server_set_fill")

    def _check(self, rc: int, what: str):
        if rc != OK:
            msg = _lib.mpmx_last_error(self.ctx._h)
            raise MpmxError(rc, f"{what}: {msg.decode() if msg else ''}")

    def clock(self) -> float:
        return float(_lib.mpmx_server_clock(self._h))

    def submit(self, scene: dict, nsteps: int, precision: int = FP32, tag: int = 0, borrow: bool = False,
               out: bool = False) -> int:
        """Queue a request.  borrow: the server keeps the particle arrays by
        pointer (this object holds them until the completion is polled); out:
        the final state goes to arrays allocated here (returned by poll)
        instead of the server's own."""
        keep = []
        n = len(scene["x"])
        arrs = [_host_f64(scene["x"], (n, 3)), _host_f64(scene["v"], (n, 3)),
                _host_f64(scene["stress"], (n, 6)) if scene.get("stress") is not None else None,
                _host_f64(scene["vol"], (n,)), _host_f64(scene["mass"], (n,))]
        parts = Particles()
        parts.size = ctypes.sizeof(Particles)
        parts.mem = MEM_HOST
        parts.n = n
        parts.x, parts.v, parts.stress, parts.vol, parts.mass = [a.ctypes.data if a is not None else None
                                                                 for a in arrs]
        mesh = _mesh(scene["mesh"])
        mat = _material(scene["material"])
        cbc = _bc(scene["bc"], keep)
        sch = _scheme(scene["scheme"], precision, SORT_ON_DEMAND)
        outs, pout = None, None
        if out:
            outs = {"x": np.empty((n, 3)), "v": np.empty((n, 3)), "stress": np.empty((n, 6)), "vol": np.empty(n)}
            po = ParticlesOut()
            po.size = ctypes.sizeof(ParticlesOut)
            po.mem = MEM_HOST
            po.x, po.v, po.stress, po.vol = [outs[k].ctypes.data for k in ("x", "v", "stress", "vol")]
            po.cell = None
            pout = ctypes.pointer(po)
        req = Request(ctypes.sizeof(Request), REQ_BORROW if borrow else 0, ctypes.pointer(mesh),
                      ctypes.pointer(mat), ctypes.pointer(cbc), ctypes.pointer(sch), ctypes.pointer(parts),
                      int(nsteps), int(tag), pout)
        rid = _u64()
        self._check(_lib.mpmx_server_submit(self._h, ctypes.byref(req), ctypes.byref(rid)), "server_submit")
        if borrow or out:
            self._held[int(rid.value)] = (arrs if borrow else None, outs)
        return int(rid.value)

    def tick(self) -> tuple[int, int]:
        r, q = ctypes.c_int(), ctypes.c_int()
        self._check(_lib.mpmx_server_tick(self._h, ctypes.byref(r), ctypes.byref(q)), "server_tick")
        return r.value, q.value

    def poll(self, max_n: int = 64, copy_state: bool = True) -> list[dict]:
        """Finished requests (oldest first); their host arrays are copied
        out (or skipped with copy_state=False) and released."""
        buf = (Completion * max_n)()
        n = ctypes.c_int()
        self._check(_lib.mpmx_server_poll(self._h, buf, max_n, ctypes.byref(n)), "server_poll")
        out = []
        for c in buf[:n.value]:
            d = {"request": int(c.request), "tag": int(c.tag), "status": int(c.status), "n": int(c.n),
                 "steps_done": int(c.steps_done), "t_submit": c.t_submit, "t_admit": c.t_admit,
                 "t_done": c.t_done}
            _, outs = self._held.pop(int(c.request), (None, None))
            if copy_state and outs is not None and c.status == OK:
                d.update(outs)
            elif copy_state and c.n > 0 and c.x:
                k = int(c.n)
                d["x"] = np.ctypeslib.as_array(c.x, shape=(k, 3)).copy()
                d["v"] = np.ctypeslib.as_array(c.v, shape=(k, 3)).copy()
                d["stress"] = np.ctypeslib.as_array(c.stress, shape=(k, 6)).copy()
                d["vol"] = np.ctypeslib.as_array(c.vol, shape=(k,)).copy()
            self._check(_lib.mpmx_server_release(self._h, c.request), "server_release")
            out.append(d)
        return out

    def close(self):
        if self._h:
            _lib.mpmx_server_destroy(self._h)
            self._h = _vp()
        getattr(self, "_held", {}).clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
