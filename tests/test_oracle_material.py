"""Pins of the oracle's constitutive update (the Material role of the code
overview: updated stress for a strain increment).  Linear elasticity is
checked against the inverse of the textbook compliance matrix; the
Drucker-Prager cone constants against Mohr-Coulomb states on the matching
meridian; the return map against consistency, the flow rule and the apex."""
import math

import numpy as np
import pytest

import oracle
from paper_1909_13380_amd import scenes

E, NU = 10.0e6, 0.3


def compliance(E, nu):
    """Voigt compliance with engineering shear: eps = C sigma."""
    C = np.zeros((6, 6))
    for a in range(3):
        for b in range(3):
            C[a, b] = 1.0 / E if a == b else -nu / E
    G = E / (2 * (1 + nu))
    for a in range(3, 6):
        C[a, a] = 1.0 / G
    return C


def test_linear_elastic_increment_is_inverse_compliance():
    mat = scenes.elastic(E=E, nu=NU)
    D = np.linalg.inv(compliance(E, NU))
    rng = np.random.default_rng(0)
    for _ in range(50):
        deps = rng.normal(scale=1e-4, size=6)
        sig0 = rng.normal(scale=1e3, size=6)
        new, kind = oracle.constitutive(mat, deps, sig0)
        assert kind == 0
        np.testing.assert_allclose(new - sig0, D @ deps, rtol=1e-12, atol=1e-9)


def test_linear_elastic_uniaxial_strain_and_shear():
    mat = scenes.elastic(E=E, nu=NU)
    e = 1e-5
    new, _ = oracle.constitutive(mat, [0, 0, e, 0, 0, 0], np.zeros(6))
    M = E * (1 - NU) / ((1 + NU) * (1 - 2 * NU))      # constrained modulus
    lam = E * NU / ((1 + NU) * (1 - 2 * NU))
    assert new[2] == pytest.approx(M * e, rel=1e-13)
    assert new[0] == pytest.approx(lam * e, rel=1e-13) and new[1] == pytest.approx(lam * e, rel=1e-13)
    new, _ = oracle.constitutive(mat, [0, 0, 0, 0, e, 0], np.zeros(6))   # engineering shear gamma_yz
    assert new[4] == pytest.approx(E / (2 * (1 + NU)) * e, rel=1e-13)
    assert np.count_nonzero(new) == 1


def principal_to_voigt(s1, s2, s3, rng):
    """A stress with principal values s1, s2, s3 in a random orientation."""
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    S = Q @ np.diag([s1, s2, s3]) @ Q.T
    return np.array([S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[1, 2], S[0, 2]])


def dp_f(sig, eta, xi, c):
    p = sig[:3].mean()
    s = sig.copy()
    s[:3] -= p
    J2 = 0.5 * (s[:3] ** 2).sum() + (s[3:] ** 2).sum()
    return math.sqrt(J2) + eta * p - xi * c


@pytest.mark.parametrize("phi_deg,c", [(30.0, 0.0), (30.0, 5e3), (20.0, 2e3), (40.0, 1e3)])
def test_dp_cones_touch_mohr_coulomb_on_their_meridians(phi_deg, c):
    """Outer cone: through the Mohr-Coulomb triaxial-compression meridian
    (two larger principal stresses equal); inner cone: through the extension
    meridian (two smaller equal).  Mohr-Coulomb, tension positive, with
    s1 >= s2 >= s3: (s1 - s3) + (s1 + s3) sin(phi) - 2 c cos(phi) = 0."""
    rng = np.random.default_rng(1)
    phi = math.radians(phi_deg)
    sp, cp = math.sin(phi), math.cos(phi)
    for cone, meridian in ((scenes.DP_OUTER, "compression"), (scenes.DP_INNER, "extension")):
        mat = scenes.drucker_prager(phi_deg=phi_deg, c=c, cone=cone)
        eta, xi, _ = oracle.dp_coefficients(mat)
        for s3 in (-1e5, -3e4, -1e4):
            s1 = (2 * c * cp + s3 * (1 - sp)) / (1 + sp)   # on the MC surface
            if meridian == "compression":
                sig = principal_to_voigt(s1, s1, s3, rng)
            else:
                sig = principal_to_voigt(s1, s3, s3, rng)
            assert dp_f(sig, eta, xi, c) == pytest.approx(0.0, abs=1e-9 * abs(s3))


def test_dp_plane_strain_cone_limits():
    # phi -> 0: plane-strain cone is sqrt(J2) = c (pure shear at yield, Tresca);
    # outer cone is sqrt(J2) = 2c/sqrt(3) (circumscribes Tresca).
    eta, xi, _ = oracle.dp_coefficients(scenes.drucker_prager(phi_deg=0.0, c=1.0, cone=scenes.DP_PLANE_STRAIN))
    assert eta == pytest.approx(0.0, abs=1e-15) and xi == pytest.approx(1.0, rel=1e-14)
    eta, xi, _ = oracle.dp_coefficients(scenes.drucker_prager(phi_deg=0.0, c=1.0, cone=scenes.DP_OUTER))
    assert eta == pytest.approx(0.0, abs=1e-15) and xi == pytest.approx(2 / math.sqrt(3), rel=1e-14)


def random_trials(rng, count):
    out = []
    for _ in range(count):
        p = rng.uniform(-5e4, 1e4)
        s = rng.normal(scale=rng.uniform(1e2, 4e4), size=6)
        s[:3] -= s[:3].mean()
        sig = s.copy()
        sig[:3] += p
        out.append(sig)
    return out


@pytest.mark.parametrize("psi_deg,c", [(0.0, 0.0), (0.0, 3e3), (10.0, 3e3), (30.0, 1e3)])
def test_dp_return_consistency_and_flow_rule(psi_deg, c):
    """Return to the cone: f(new) = 0; sigma_trial - sigma_new is the elastic
    image of dgamma * dg/dsigma with g = sqrt(J2) + eta_bar p, i.e. a
    deviatoric part G dgamma s*/sqrt(J2*) along the trial deviator and a
    pressure drop K eta_bar dgamma, with one dgamma >= 0 for both."""
    mat = scenes.drucker_prager(phi_deg=30.0, psi_deg=psi_deg, c=c)
    eta, xi, etab = oracle.dp_coefficients(mat)
    G = E / (2 * (1 + NU))
    K = E / (3 * (1 - 2 * NU))
    rng = np.random.default_rng(2)
    kinds = set()
    for trial in random_trials(rng, 400):
        new, kind = oracle.constitutive(mat, np.zeros(6), trial)
        kinds.add(kind)
        ft = dp_f(trial, eta, xi, c)
        if ft <= 0:
            assert kind == 0
            np.testing.assert_array_equal(new, trial)
            continue
        scale = max(abs(trial).max(), 1.0)
        if kind == 1:
            assert dp_f(new, eta, xi, c) == pytest.approx(0.0, abs=1e-10 * scale)
            pt, pn = trial[:3].mean(), new[:3].mean()
            st, sn = trial.copy(), new.copy()
            st[:3] -= pt
            sn[:3] -= pn
            qt = math.sqrt(0.5 * (st[:3] ** 2).sum() + (st[3:] ** 2).sum())
            dgam_dev = (qt - math.sqrt(0.5 * (sn[:3] ** 2).sum() + (sn[3:] ** 2).sum())) / G
            np.testing.assert_allclose(st - sn, G * dgam_dev * st / qt, atol=1e-9 * scale)
            assert dgam_dev >= 0
            if etab > 0:
                assert (pt - pn) / (K * etab) == pytest.approx(dgam_dev, rel=1e-9)
            else:
                assert pn == pytest.approx(pt, abs=1e-10 * scale)
        else:
            assert kind == 2
            np.testing.assert_allclose(new[3:], 0.0, atol=0)
            np.testing.assert_allclose(new[:3], xi * c / eta, rtol=1e-13, atol=1e-12)
    assert {0, 1, 2} <= kinds


def test_dp_cohesionless_closed_form_cases():
    mat = scenes.drucker_prager(phi_deg=30.0)
    eta, xi, etab = oracle.dp_coefficients(mat)
    assert eta == pytest.approx(6 * 0.5 / (math.sqrt(3) * 2.5), rel=1e-14)
    assert etab == pytest.approx(0.0, abs=1e-16)
    # hydrostatic tension is cut to zero stress; hydrostatic compression is elastic
    new, kind = oracle.constitutive(mat, np.zeros(6), [1e3, 1e3, 1e3, 0, 0, 0])
    assert kind == 2 and np.all(new == 0)
    new, kind = oracle.constitutive(mat, np.zeros(6), [-1e3, -1e3, -1e3, 0, 0, 0])
    assert kind == 0
    # pure shear at zero pressure returns to the apex (zero stress)
    new, kind = oracle.constitutive(mat, np.zeros(6), [0, 0, 0, 1e3, 0, 0])
    assert np.allclose(new, 0.0, atol=1e-12)


@pytest.mark.parametrize("phi_deg,c", [(30.0, 0.0), (30.0, 4e3), (20.0, 1e3), (40.0, 2e3)])
def test_dp_plane_strain_cone_reproduces_mohr_coulomb_in_plane_strain(phi_deg, c):
    """The plane-strain cone is the one whose associated flow, with no plastic
    strain out of the plane, yields exactly on the Mohr-Coulomb line of the
    in-plane principal stresses s1 = m + t, s3 = m - t:
    t = c cos(phi) - m sin(phi) (tension positive).  With the out-of-plane
    stress z = m + d, sqrt(J2) = sqrt(t^2 + d^2 / 3), and zero out-of-plane
    flow, d/s_zz-direction: (2/3) d = -(2/3) eta sqrt(J2), which fixes
    d = -eta t / sqrt(1 - eta^2 / 3).  Such states must sit on the oracle's
    cone for every m and c: a state a hair inside stays elastic, a hair
    outside returns.  A wrong coefficient in eta or xi moves f off zero."""
    rng = np.random.default_rng(7)
    phi = math.radians(phi_deg)
    mat = scenes.drucker_prager(phi_deg=phi_deg, psi_deg=phi_deg, c=c, cone=scenes.DP_PLANE_STRAIN)
    eta, xi, etab = oracle.dp_coefficients(mat)
    assert etab == pytest.approx(eta, rel=1e-15)          # associated: psi = phi
    for m in (-8e4, -2e4, -5e3):
        t = c * math.cos(phi) - m * math.sin(phi)
        d = -eta * t / math.sqrt(1.0 - eta * eta / 3.0)
        sig = principal_to_voigt(m + t, m + d, m - t, rng)
        scale = abs(m) + c
        assert dp_f(sig, eta, xi, c) == pytest.approx(0.0, abs=1e-10 * scale)
        # the deviator's out-of-plane component equals the flow condition
        for f, kind in ((1.0 - 1e-6, 0), (1.0 + 1e-6, 1)):
            p = sig[:3].mean()
            trial = sig.copy()
            trial[:3] -= p
            trial *= f
            trial[:3] += p
            _, got = oracle.constitutive(mat, np.zeros(6), trial)
            assert got == kind, (m, f)


def test_dp_cone_constants_at_thirty_degrees():
    """At phi = 30 deg: outer eta = 2 sqrt(3)/5 = 0.69282 (M_c = 1.2); inner
    eta = 6 (1/2) / (sqrt(3) 3.5) = 0.49487; plane strain eta =
    3 tan(30) / sqrt(13) = 0.48038 (tan^2 = 1/3)."""
    want = {scenes.DP_OUTER: 0.69282, scenes.DP_INNER: 0.49487, scenes.DP_PLANE_STRAIN: 0.48038}
    for cone, eta_w in want.items():
        eta, xi, _ = oracle.dp_coefficients(scenes.drucker_prager(phi_deg=30.0, cone=cone))
        assert eta == pytest.approx(eta_w, abs=5e-6), cone
    eta, xi, _ = oracle.dp_coefficients(scenes.drucker_prager(phi_deg=30.0, cone=scenes.DP_PLANE_STRAIN))
    assert xi == pytest.approx(3.0 / math.sqrt(13.0), rel=1e-14)
