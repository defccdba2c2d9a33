"""Pins for the oracle's BSDF sampling (Sec. 3.1: diffuse, mirror, dielectric
surfaces).  Fresnel is checked against the angle form of the Fresnel
equations (an independent formula), refraction against Snell's law, the
orthonormal basis against orthonormality, cosine sampling by chi^2."""
import numpy as np
from scipy import stats

import oracle as O


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


def _fresnel_angles(ti, n1, n2):
    """Unpolarised reflectance from the angle form (Born & Wolf)."""
    st = n1 / n2 * np.sin(ti)
    if st >= 1:
        return 1.0
    tt = np.arcsin(st)
    if ti == 0:
        return ((n1 - n2) / (n1 + n2)) ** 2
    rs = (np.sin(ti - tt) / np.sin(ti + tt)) ** 2
    rp = (np.tan(ti - tt) / np.tan(ti + tt)) ** 2
    return 0.5 * (rs + rp)


def test_fresnel_normal_incidence():
    assert abs(O.fresnel_dielectric(1.0, 1.0, 1.5) - 0.04) < 2e-8
    assert abs(O.fresnel_dielectric(1.0, 1.5, 1.0) - 0.04) < 2e-8


def test_fresnel_matches_angle_form():
    for n1, n2 in ((1.0, 1.5), (1.5, 1.0), (1.0, 1.33)):
        for ti in np.linspace(1e-3, np.pi / 2 - 1e-3, 300):
            f = O.fresnel_dielectric(np.float32(np.cos(ti)), n1, n2)
            assert abs(f - _fresnel_angles(ti, n1, n2)) < 3e-6, (n1, n2, ti)


def test_fresnel_tir_and_reciprocity():
    crit = np.arcsin(1 / 1.5)
    for ti in np.linspace(crit + 1e-3, np.pi / 2, 50):
        assert O.fresnel_dielectric(np.cos(ti), 1.5, 1.0) == 1.0
    for ti in np.linspace(0.01, 1.5, 40):
        tt = np.arcsin(np.sin(ti) / 1.5)
        a = O.fresnel_dielectric(np.cos(ti), 1.0, 1.5)
        b = O.fresnel_dielectric(np.cos(tt), 1.5, 1.0)
        assert abs(a - b) < 1e-5


def test_refraction_obeys_snell_and_reflection_the_mirror_law():
    rng = np.random.default_rng(0)
    n = np.array([0, 0, 1], np.float32)
    nr = nt = 0
    for _ in range(3000):
        d = _unit(rng.normal(size=3))
        u = np.float32(rng.random())
        out, refl = O.dielectric_scatter(d.astype(np.float32), n, 1.5, u)
        d32 = d.astype(np.float32).astype(np.float64)
        entering = d32[2] < 0
        o = out.astype(np.float64)
        assert abs(np.linalg.norm(o) - 1) < 1e-5
        # coplanar with d and n
        assert abs(np.dot(np.cross(d32, [0, 0, 1]), o)) < 1e-5
        sin_i = np.linalg.norm(d32[:2])
        if refl:
            nr += 1
            assert np.allclose(o, [d32[0], d32[1], -d32[2]], atol=1e-6)
        else:
            nt += 1
            eta = 1 / 1.5 if entering else 1.5
            assert abs(np.linalg.norm(o[:2]) - eta * sin_i) < 2e-6
            assert np.sign(o[2]) == np.sign(d32[2])  # transmitted: same side as d
    assert nr > 100 and nt > 1000


def test_reflect_fraction_equals_fresnel():
    n = np.array([0, 0, 1], np.float32)
    for ti in (0.2, 0.8, 1.3):
        d = np.array([np.sin(ti), 0, -np.cos(ti)], np.float32)
        us = (np.arange(4096, dtype=np.float64) + 0.5) / 4096
        frac = np.mean([O.dielectric_scatter(d, n, 1.5, np.float32(u))[1] for u in us])
        assert abs(frac - O.fresnel_dielectric(np.cos(ti), 1.0, 1.5)) < 1.0 / 4096 + 1e-6


def test_onb_orthonormal():
    rng = np.random.default_rng(1)
    ns = [_unit(rng.normal(size=3)) for _ in range(2000)] + [
        np.array([0, 0, 1.0]), np.array([0, 0, -1.0]), np.array([1.0, 0, 0]), np.array([0, 1.0, 0]),
        _unit([1e-4, 0, -1])]
    for n in ns:
        n32 = n.astype(np.float32)
        t, b = O.onb(n32)
        t, b, n64 = t.astype(np.float64), b.astype(np.float64), n32.astype(np.float64)
        for a in (t, b):
            assert abs(np.linalg.norm(a) - 1) < 2e-6
            assert abs(np.dot(a, n64)) < 2e-6
        assert abs(np.dot(t, b)) < 2e-6
        assert np.allclose(np.cross(t, b), n64, atol=3e-6)  # right-handed


def test_cosine_sampling_chi2():
    rng = np.random.default_rng(2)
    n = _unit([0.3, -0.5, 0.8]).astype(np.float32)
    N = 60000
    u = rng.random((N, 2), dtype=np.float32)
    cos = np.empty(N)
    phi_ok = 0
    for i in range(N):
        d = O.cosine_sample(n, u[i, 0], u[i, 1]).astype(np.float64)
        cos[i] = np.dot(d, n)
        assert cos[i] >= -1e-6
    # cos(theta)^2 is uniform on [0,1] under a cosine-weighted density
    bins = 40
    h, _ = np.histogram(np.clip(cos, 0, 1) ** 2, bins=bins, range=(0, 1))
    chi2 = ((h - N / bins) ** 2 / (N / bins)).sum()
    assert stats.chi2.sf(chi2, bins - 1) > 1e-4


def test_cosine_sample_closed_form_points():
    n = np.array([0, 0, 1], np.float32)
    assert O.cosine_sample(n, 0.0, 0.3).tolist() == [0.0, 0.0, 1.0]
    d = O.cosine_sample(n, 0.25, 0.0)  # r = 0.5, phi = 0
    t, b = O.onb(n)
    assert np.allclose(d, 0.5 * t + np.sqrt(0.75) * n, atol=1e-7)
