"""The C ABI library without a GPU: it loads, exports every function that
include/mpmx.h declares, its descriptor layouts agree with what a C compiler
makes of the header, and the pure sizing call works.  No compute runs."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def mpmx():
    from paper_1909_13380_amd import mpmx
    return mpmx


def test_library_exports_every_declared_function(mpmx):
    names = mpmx.declared_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(mpmx.LIBPATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert mpmx.version() == 4


def test_header_constants_match_the_binding(mpmx):
    # the error bits a scene can report, and the tuning threshold, as the
    # header declares them
    text = open(mpmx.HEADER).read()
    import re
    bits = dict((k, int(v)) for k, v in re.findall(r"MPMX_ERRBIT_(\w+) = (\d+)u", text))
    assert bits == {"OUT_OF_MESH": 1, "NONFINITE": 2, "TILE": 4, "SORT": 8}
    assert (mpmx.ERRBIT_OUT_OF_MESH, mpmx.ERRBIT_NONFINITE, mpmx.ERRBIT_TILE, mpmx.ERRBIT_SORT) == (1, 2, 4, 8)
    m = re.search(r"#define MPMX_TUNE_MIN_STEPS (\d+)", text)
    assert int(m.group(1)) == mpmx.TUNE_MIN_STEPS


def test_descriptor_layouts_match_the_c_header(mpmx, tmp_path):
    structs = {"mpmx_mesh": mpmx.Mesh, "mpmx_material": mpmx.Material, "mpmx_bc": mpmx.Bc,
               "mpmx_scheme": mpmx.Scheme, "mpmx_particles": mpmx.Particles,
               "mpmx_particles_out": mpmx.ParticlesOut, "mpmx_stats": mpmx.Stats,
               "mpmx_request": mpmx.Request, "mpmx_completion": mpmx.Completion}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mpmx.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            if field != "pad_":
                lines.append(f'printf("{cname}.{field} %zu\\n", offsetof({cname}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True, check=True)
               .stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            if field != "pad_":
                assert int(got[f"{cname}.{field}"]) == getattr(py, field).offset, f"{cname}.{field}"


def test_scene_bytes_is_pure_and_grows_with_size(mpmx):
    from paper_1909_13380_amd import scenes
    sc = scenes.c1()
    b32 = mpmx.scene_bytes(sc, mpmx.FP32)
    b64 = mpmx.scene_bytes(sc, mpmx.FP64)
    assert 0 < b32 < b64
    assert mpmx.scene_bytes(sc, mpmx.FP32, n_particles=2 * len(sc["x"])) > b32
    # the large column: ~160 B per particle, two node buffers of 32 B per node,
    # 8 B per sort key
    col = {"mesh": {"n": (256, 128, 160), "origin": (0, 0, 0), "h": 0.01}, "scheme": scenes.scheme(2e-5)}
    b = mpmx.scene_bytes(col, mpmx.FP32, n_particles=2_097_152)
    assert 500e6 < b < 900e6
    # MUSL scenes add one array of remapped nodal momenta (3 components)
    nn = 257 * 129 * 161
    for prec, R in ((mpmx.FP32, 4), (mpmx.FP64, 8)):
        usl = dict(col, scheme=dict(col["scheme"], algo=mpmx.USL))
        musl = dict(col, scheme=dict(col["scheme"], algo=mpmx.MUSL))
        extra = mpmx.scene_bytes(musl, prec, n_particles=1000) - mpmx.scene_bytes(usl, prec, n_particles=1000)
        assert extra == (3 * R * nn + 255) // 256 * 256
    with pytest.raises(mpmx.MpmxError):
        mpmx.scene_bytes(dict(col, scheme=dict(col["scheme"], algo=3)), mpmx.FP32, n_particles=10)


def test_invalid_descriptors_are_rejected(mpmx):
    from paper_1909_13380_amd import scenes
    sc = scenes.c1()
    bad = dict(sc, mesh={"n": (0, 4, 4), "origin": (0, 0, 0), "h": 0.1})
    with pytest.raises(mpmx.MpmxError) as e:
        mpmx.scene_bytes(bad)
    assert e.value.code == mpmx.E_INVALID_ARG
    bad = dict(sc, scheme=dict(sc["scheme"], dt=-1.0))
    with pytest.raises(mpmx.MpmxError):
        mpmx.scene_bytes(bad)
    with pytest.raises(mpmx.MpmxError):
        mpmx.scene_bytes(sc, n_particles=-5)


def test_context_creation_fails_cleanly_without_a_gpu(mpmx):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(mpmx.MpmxError) as e:
        mpmx.Context(0)
    assert e.value.code == mpmx.E_HIP


def test_server_queue_without_a_gpu(mpmx):
    """The server's host side (copying requests, budget check, queue,
    polling) needs no device: a server on a placeholder context accepts and
    queues requests, rejects one that can never fit its budget, and has
    nothing to report before a tick.  (Ticks need a GPU.)"""
    import ctypes
    from paper_1909_13380_amd import scenes
    sc = scenes.c1()
    need = mpmx.scene_bytes(sc, mpmx.FP32)
    h = ctypes.c_void_p()
    placeholder = ctypes.c_void_p(1)            # never dereferenced by submit/poll
    assert mpmx._lib.mpmx_server_create(placeholder, 0, 16, ctypes.byref(h)) == mpmx.E_INVALID_ARG
    assert mpmx._lib.mpmx_server_create(placeholder, need, 0, ctypes.byref(h)) == mpmx.E_INVALID_ARG
    assert mpmx._lib.mpmx_server_create(placeholder, need, 16, ctypes.byref(h)) == mpmx.OK
    assert mpmx._lib.mpmx_server_set_fill(h, -1) == mpmx.E_INVALID_ARG
    assert mpmx._lib.mpmx_server_set_fill(None, 100) == mpmx.E_INVALID_ARG
    assert mpmx._lib.mpmx_server_set_fill(h, 0) == mpmx.OK
    f, d = ctypes.c_uint64(0), ctypes.c_int(0)
    assert mpmx._lib.mpmx_fence_record(None, ctypes.byref(f)) == mpmx.E_INVALID_ARG
    assert mpmx._lib.mpmx_fence_wait(None, 1, 0, ctypes.byref(d)) == mpmx.E_INVALID_ARG
    assert mpmx._lib.mpmx_fence_release(None, 1) == mpmx.E_INVALID_ARG

    class _Ctx:
        _h = placeholder
    srv = mpmx.Server.__new__(mpmx.Server)
    srv.ctx, srv._h = _Ctx(), h
    srv._check = lambda rc, what: (_ for _ in ()).throw(mpmx.MpmxError(rc, what)) if rc else None
    ids = [srv.submit(sc, 10, tag=7), srv.submit(sc, 0)]
    assert ids == [1, 2]
    big = dict(sc, x=np.concatenate([sc["x"]] * 2), v=np.concatenate([sc["v"]] * 2),
               vol=np.concatenate([sc["vol"]] * 2), mass=np.concatenate([sc["mass"]] * 2), stress=None)
    with pytest.raises(mpmx.MpmxError) as e:
        srv.submit(big, 10)
    assert e.value.code == mpmx.E_BUDGET
    with pytest.raises(mpmx.MpmxError) as e:
        srv.submit(sc, -1)
    assert e.value.code == mpmx.E_INVALID_ARG
    assert srv.poll() == []
    assert mpmx._lib.mpmx_server_release(h, ids[0]) == mpmx.E_NOT_FOUND
    t = srv.clock()
    assert 0.0 <= t < 60.0
    srv.close()
