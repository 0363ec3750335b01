"""Pins of the oracle's isoparametric mesh (isoparametric-mesh section: cells
that are trilinear images of the natural cube, points located by inverting
that map with Newton-Raphson from an affine initial guess).

What fixes it, beyond the oracle's own formulas:
  - a uniform grid given as a node list must behave exactly as the uniform
    mesh (cells, weights, gradients, whole steps);
  - on affine (parallelepiped) cells the inverse map is the affine inverse,
    which the affine initial guess already is;
  - points made by the forward map at known natural coordinates of a known
    cell (written out here with numpy, independently) are found there;
  - partition of unity, zero gradient sum and linear completeness
    (sum_I X_I (x) grad N_I = identity) on distorted cells;
  - a free body moved rigidly (rotated mesh, particles, velocities, stress
    and gravity) moves with its rotated image, step for step;
  - free fall on a distorted mesh keeps its discrete closed form."""
import math

import numpy as np
import pytest

import oracle
from paper_1909_13380_amd import scenes


def trilinear_point(X8, xi):
    """x = sum_q N_q(xi) X_q, node q = i + 2j + 4k at corner (i, j, k)."""
    s = np.array([[(q & 1) * 2 - 1, ((q >> 1) & 1) * 2 - 1, (q >> 2) * 2 - 1] for q in range(8)], dtype=float)
    N = 0.125 * np.prod(1.0 + s * np.asarray(xi)[None, :], axis=1)
    return N @ X8


def corners(mesh, c):
    nx, ny = mesh["n"][0] + 1, mesh["n"][1] + 1
    X = np.asarray(mesh["node_x"])
    return np.array([X[(c[0] + (q & 1)) + nx * ((c[1] + ((q >> 1) & 1)) + ny * (c[2] + (q >> 2)))]
                     for q in range(8)])


def random_rotation(seed):
    Q, _ = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    return Q if np.linalg.det(Q) > 0 else -Q


def test_uniform_grid_as_node_list_equals_uniform_mesh():
    sc = scenes.random_block(n_cells=(5, 4, 3), mesh_cells=(9, 8, 6), seed=61, stress_scale=2e3)
    iso = dict(sc, mesh=dict(sc["mesh"], node_x=scenes.uniform_nodes(sc["mesh"])))
    np.testing.assert_array_equal(oracle.locate(iso["mesh"], sc["x"]), oracle.locate(sc["mesh"], sc["x"]))
    for p in range(0, len(sc["x"]), 37):
        n0, N0, d0 = oracle.shape(sc["mesh"], 0, sc["x"][p])
        n1, N1, d1 = oracle.shape(iso["mesh"], 0, sc["x"][p])
        np.testing.assert_array_equal(n0, n1)
        np.testing.assert_allclose(N1, N0, rtol=0, atol=1e-14)
        np.testing.assert_allclose(d1, d0, rtol=0, atol=1e-12 * np.abs(d0).max())
    a, b = oracle.run(sc, 6), oracle.run(iso, 6)
    for k in ("x", "v", "stress", "vol"):
        scale = np.abs(a[k] - (sc[k] if k == "x" else 0)).max() or 1.0
        np.testing.assert_allclose(b[k], a[k], rtol=0, atol=1e-11 * scale)


def test_affine_cells_invert_exactly_from_the_affine_guess():
    mesh = {"n": (4, 3, 5), "origin": (0.1, -0.2, 0.3), "h": 0.05}
    A = np.array([[1.1, 0.3, -0.2], [0.1, 0.9, 0.25], [-0.15, 0.2, 1.2]])
    b = np.array([0.7, -0.4, 1.3])
    mesh["node_x"] = scenes.uniform_nodes(mesh) @ A.T + b
    rng = np.random.default_rng(62)
    for _ in range(60):
        c = [int(rng.integers(0, m)) for m in mesh["n"]]
        xi = rng.uniform(-1, 1, size=3)
        u = np.asarray(mesh["origin"]) + mesh["h"] * (np.asarray(c) + (xi + 1) / 2)   # reference point
        x = A @ u + b
        got, it = oracle.iso_natural(mesh, c, x)
        np.testing.assert_allclose(got, xi, rtol=0, atol=1e-12)
        assert it <= 2, it      # the first correction already vanishes to rounding
        cell = oracle.locate(mesh, x[None])[0]
        assert cell == c[0] + mesh["n"][0] * (c[1] + mesh["n"][1] * c[2])


@pytest.mark.parametrize("amp", [0.15, 0.3])
def test_points_made_by_the_forward_map_are_found_where_they_were_made(amp):
    base = scenes.random_block(n_cells=(4, 4, 3), mesh_cells=(8, 7, 6), seed=63)
    mesh = scenes.distort(base, amp=amp, seed=64)["mesh"]
    rng = np.random.default_rng(65)
    pts, want_c, want_xi = [], [], []
    for _ in range(300):
        c = [int(rng.integers(0, m)) for m in mesh["n"]]
        xi = rng.uniform(-0.995, 0.995, size=3)
        pts.append(trilinear_point(corners(mesh, c), xi))
        want_c.append(c[0] + mesh["n"][0] * (c[1] + mesh["n"][1] * c[2]))
        want_xi.append((c, xi))
    got = oracle.locate(mesh, np.array(pts))
    np.testing.assert_array_equal(got, want_c)
    for p, (c, xi) in zip(pts, want_xi):
        g, it = oracle.iso_natural(mesh, c, p)
        np.testing.assert_allclose(g, xi, rtol=0, atol=1e-12)
        assert it < 50
    # outside the mesh's box: no cell holds the point
    with pytest.raises(oracle.OracleError) as e:
        oracle.locate(mesh, np.array([[-1.0, 0.1, 0.1]]))
    assert e.value.code == oracle.E_OUT_OF_MESH


def test_shape_functions_on_distorted_cells():
    base = scenes.random_block(n_cells=(4, 4, 3), mesh_cells=(8, 7, 6), seed=66)
    sc = scenes.distort(base, amp=0.3, seed=67)
    X = np.asarray(sc["mesh"]["node_x"])
    for p in range(0, len(sc["x"]), 7):
        xp = sc["x"][p]
        node, N, dN = oracle.shape(sc["mesh"], 0, xp)
        assert len(node) == 8
        assert abs(N.sum() - 1.0) < 1e-14
        np.testing.assert_allclose(dN.sum(axis=0), 0.0, atol=1e-11 * np.abs(dN).max())
        np.testing.assert_allclose(N @ X[node], xp, rtol=0, atol=1e-13)
        # linear completeness: the gradient of the interpolated position is I
        np.testing.assert_allclose(X[node].T @ dN, np.eye(3), rtol=0, atol=1e-12)


def test_rotated_free_body_moves_with_its_image():
    sc = scenes.free_body(v0=(0.3, -0.2, 0.1), cells=(3, 3, 2), mesh_cells=(9, 9, 8))
    rng = np.random.default_rng(68)
    sc["v"] = sc["v"] + rng.uniform(-0.05, 0.05, size=sc["v"].shape)     # the body deforms
    sc["stress"] = rng.uniform(-1e3, 1e3, size=sc["stress"].shape)
    R, b = random_rotation(69), np.array([1.3, -0.7, 2.1])
    rot = scenes.rotate(sc, R, b)
    n = 12
    a, r = oracle.run(sc, n), oracle.run(rot, n)
    np.testing.assert_allclose(r["x"], a["x"] @ R.T + b, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["v"], a["v"] @ R.T, rtol=0, atol=1e-11 * np.abs(a["v"]).max())
    want = scenes.rotate(dict(sc, stress=a["stress"]), R)["stress"]
    np.testing.assert_allclose(r["stress"], want, rtol=0, atol=1e-9 * np.abs(a["stress"]).max())
    np.testing.assert_allclose(r["vol"], a["vol"], rtol=1e-12)


def test_free_fall_on_a_distorted_mesh():
    sc = scenes.distort(scenes.free_body(v0=(0.3, -0.2, 0.1), cells=(3, 3, 3), mesh_cells=(9, 9, 9)),
                        amp=0.25, seed=70)
    sc["scheme"]["mass_eps_rel"] = 0.0
    v0 = sc["v"][0]
    g = np.array(scenes.GRAVITY)
    dt = sc["scheme"]["dt"]
    n = 20
    out = oracle.run(sc, n)
    np.testing.assert_allclose(out["v"], np.broadcast_to(v0 + n * g * dt, out["v"].shape), rtol=1e-12)
    np.testing.assert_allclose(out["x"] - sc["x"],
                               np.broadcast_to(n * dt * v0 + g * dt * dt * n * (n + 1) / 2, sc["x"].shape),
                               rtol=1e-10)
    assert np.abs(out["stress"]).max() < 1e-7
