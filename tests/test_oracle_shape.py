"""Pins of the oracle's particle location and shape functions against
definitions that do not use the oracle's own formulas: the global tent
function of a node, numerical averaging of that tent over a particle domain
(uGIMP), brute-force point-in-box search, partition of unity and finite
differences.  (Code overview: linear/GIMP mapping functions on hexahedra;
active cells.)"""
import numpy as np
import pytest

import oracle

# dyadic origin and spacing: points placed on cell faces are exact in binary
MESH = {"n": (5, 4, 3), "origin": (0.5, -0.25, 0.125), "h": 0.25}


def tent(r, h):
    return np.maximum(0.0, 1.0 - np.abs(r) / h)


def node_xyz(mesh, shape, I):
    g = 1 if shape == oracle.SHAPE_GIMP else 0
    n0, n1 = mesh["n"][0] + 1 + 2 * g, mesh["n"][1] + 1 + 2 * g
    i = I % n0 - g
    j = (I // n0) % n1 - g
    k = I // (n0 * n1) - g
    return np.array([i, j, k])


def random_points(mesh, rng, count, margin=0.0):
    lo = np.array(mesh["origin"]) + margin
    hi = np.array(mesh["origin"]) + np.array(mesh["n"]) * mesh["h"] - margin
    return rng.uniform(lo, hi, size=(count, 3))


def test_locate_matches_brute_force_box_search():
    rng = np.random.default_rng(0)
    h = MESH["h"]
    o = np.array(MESH["origin"])
    pts = list(random_points(MESH, rng, 300))
    # points exactly on interior cell faces belong to the upper cell (half-open cells)
    pts += [o + h * np.array([1.0, 2.0, 1.0]), o + h * np.array([0.0, 0.0, 0.0]), o + h * np.array([4.0, 3.5, 2.0])]
    pts = np.array(pts)
    cells = oracle.locate(MESH, pts)
    nx, ny, nz = MESH["n"]
    for p, c in zip(pts, cells):
        found = []
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    lo = o + h * np.array([i, j, k])
                    if np.all(p >= lo) and np.all(p < lo + h):
                        found.append(i + nx * (j + ny * k))
        assert found == [c]


def test_locate_rejects_points_outside():
    o = np.array(MESH["origin"])
    top = o + np.array(MESH["n"]) * MESH["h"]
    for bad in (o - 1e-9, np.array([top[0], o[1] + 0.1, o[2] + 0.1]), np.array([o[0] + 0.1, o[1] + 0.1, top[2] + 1.0])):
        with pytest.raises(oracle.OracleError) as e:
            oracle.locate(MESH, bad[None, :])
        assert e.value.code == oracle.E_OUT_OF_MESH


def test_linear_weights_are_global_tent_functions():
    rng = np.random.default_rng(1)
    h = MESH["h"]
    o = np.array(MESH["origin"])
    for xp in random_points(MESH, rng, 200):
        node, N, dN = oracle.shape(MESH, oracle.SHAPE_LINEAR, xp)
        assert len(node) == 8
        for I, w, g in zip(node, N, dN):
            X = o + h * node_xyz(MESH, oracle.SHAPE_LINEAR, I)
            t = tent(xp - X, h)
            assert w == pytest.approx(np.prod(t), rel=1e-13, abs=1e-15)
            # derivative of the tent product, written independently
            dt = -np.sign(xp - X) / h
            ref = np.array([dt[0] * t[1] * t[2], t[0] * dt[1] * t[2], t[0] * t[1] * dt[2]])
            np.testing.assert_allclose(g, ref, rtol=1e-12, atol=1e-12)
        # every node with a nonzero tent weight is in the support
        nx, ny, nz = MESH["n"]
        inside = 0
        for k in range(nz + 1):
            for j in range(ny + 1):
                for i in range(nx + 1):
                    if np.prod(tent(xp - (o + h * np.array([i, j, k])), h)) > 0:
                        inside += 1
        assert inside == 8


def test_linear_kronecker_delta_at_nodes():
    h = MESH["h"]
    o = np.array(MESH["origin"])
    for ijk in [(0, 0, 0), (2, 1, 1), (4, 3, 2)]:
        xp = o + h * np.array(ijk, dtype=float)
        node, N, _ = oracle.shape(MESH, oracle.SHAPE_LINEAR, xp)
        target = oracle.node_id(MESH, oracle.SHAPE_LINEAR, *ijk)
        for I, w in zip(node, N):
            assert w == pytest.approx(1.0 if I == target else 0.0, abs=1e-15)


@pytest.mark.parametrize("shape", [oracle.SHAPE_LINEAR, oracle.SHAPE_GIMP])
def test_partition_of_unity_and_zero_gradient_sum(shape):
    rng = np.random.default_rng(2)
    for xp in random_points(MESH, rng, 500):
        _, N, dN = oracle.shape(MESH, shape, xp)
        assert N.sum() == pytest.approx(1.0, abs=1e-14)
        np.testing.assert_allclose(dN.sum(axis=0), 0.0, atol=1e-12 / MESH["h"])
        assert np.all(N >= -1e-15)


@pytest.mark.parametrize("shape", [oracle.SHAPE_LINEAR, oracle.SHAPE_GIMP])
def test_gradients_match_central_differences(shape):
    rng = np.random.default_rng(3)
    h = MESH["h"]
    eps = 1e-6 * h
    for xp in random_points(MESH, rng, 100, margin=0.01):
        node, N, dN = oracle.shape(MESH, shape, xp)
        weights = dict(zip(node, N))
        for a in range(3):
            e = np.zeros(3)
            e[a] = eps
            np_, Np, _ = oracle.shape(MESH, shape, xp + e)
            nm_, Nm, _ = oracle.shape(MESH, shape, xp - e)
            wp, wm = dict(zip(np_, Np)), dict(zip(nm_, Nm))
            for I in weights:
                fd = (wp.get(I, 0.0) - wm.get(I, 0.0)) / (2 * eps)
                ref = dN[list(node).index(I), a]
                if shape == oracle.SHAPE_LINEAR:
                    # the linear hat is C0: skip if the stencil crossed a face
                    if set(np_) != set(node) or set(nm_) != set(node):
                        continue
                assert fd == pytest.approx(ref, abs=1e-6 / h)


def averaged_hat(r, h, l, m=20001):
    """Mean of the linear hat of half-width h over [r - l, r + l] (Simpson)."""
    s = np.linspace(r - l, r + l, m)
    w = np.ones(m)
    w[1:-1:2] = 4
    w[2:-1:2] = 2
    return float((tent(s, h) * w).sum() * (s[1] - s[0]) / 3.0 / (2 * l))


@pytest.mark.parametrize("l_frac", [0.25, 0.1, 0.4])
def test_gimp_weight_is_hat_averaged_over_particle_domain(l_frac):
    h = 0.5
    l = l_frac * h
    for r in np.linspace(-(h + l) * 1.05, (h + l) * 1.05, 97):
        S, dS = oracle.gimp_1d(r, h, l)
        assert S == pytest.approx(averaged_hat(r, h, l), abs=1e-9)
        d = 1e-5 * h
        fd = (averaged_hat(r + d, h, l) - averaged_hat(r - d, h, l)) / (2 * d)
        assert dS == pytest.approx(fd, abs=2e-4 / h)


def test_gimp_is_c1_at_region_joins_and_tends_to_linear():
    h, l = 1.0, 0.25
    for r0 in (l, h - l, h + l, -l, -(h - l), -(h + l)):
        a, b = oracle.gimp_1d(r0 - 1e-12, h, l), oracle.gimp_1d(r0 + 1e-12, h, l)
        assert a[0] == pytest.approx(b[0], abs=1e-10)
        assert a[1] == pytest.approx(b[1], abs=1e-10)
    for r in np.linspace(-1.2, 1.2, 49):
        S, _ = oracle.gimp_1d(r, h, 1e-7)
        assert S == pytest.approx(max(0.0, 1 - abs(r) / h), abs=1e-6)


def test_gimp_support_contains_every_nonzero_node():
    rng = np.random.default_rng(4)
    h = MESH["h"]
    l = h / 4
    o = np.array(MESH["origin"])
    nx, ny, nz = MESH["n"]
    for xp in random_points(MESH, rng, 40):
        node, N, _ = oracle.shape(MESH, oracle.SHAPE_GIMP, xp)
        assert len(node) == 27
        got = dict(zip(node, N))
        for k in range(-1, nz + 2):
            for j in range(-1, ny + 2):
                for i in range(-1, nx + 2):
                    X = o + h * np.array([i, j, k])
                    w = np.prod([oracle.gimp_1d(xp[a] - X[a], h, l)[0] for a in range(3)])
                    I = oracle.node_id(MESH, oracle.SHAPE_GIMP, i, j, k)
                    if w > 0:
                        assert got.get(I, 0.0) == pytest.approx(w, rel=1e-12)
