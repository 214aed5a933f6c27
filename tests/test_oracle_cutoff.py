"""Pins of the cut-off oracle (eq. data-part, the construction of w_cut at the
start of Section 5) against symmetry, independent one-dimensional integrals
and the reading of the printed mollifier."""
import numpy as np
import pytest
from scipy import integrate

from oracle import cutoff


def _phi(r, eps):
    q = 1.0 - (r / eps) ** 2
    return np.exp(-1.0 / q) if q > 0 else 0.0


@pytest.mark.parametrize("eps", [1.5, 2.0, 4.0])
def test_mass_against_radial_integral(eps):
    # 2D: 2 pi int r phi dr; 3D: 4 pi int r^2 phi dr (shell integrals, adaptive)
    m2 = 2 * np.pi * integrate.quad(lambda r: r * _phi(r, eps), 0, eps, epsabs=1e-14, epsrel=1e-13)[0]
    m3 = 4 * np.pi * integrate.quad(lambda r: r * r * _phi(r, eps), 0, eps, epsabs=1e-14, epsrel=1e-13)[0]
    assert cutoff.mass(eps, 2) == pytest.approx(m2, rel=1e-10)
    assert cutoff.mass(eps, 3) == pytest.approx(m3, rel=1e-10)


def _one_face_3d(u, eps):
    # int_{y1 <= u} phi / mass, the inner integral over the disc of radius
    # sqrt(eps^2 - y1^2) in polar coordinates
    def area(y1):
        rr = np.sqrt(max(eps * eps - y1 * y1, 0.0))
        return 2 * np.pi * integrate.quad(lambda p: p * _phi(np.hypot(y1, p), eps), 0, rr, epsabs=1e-14)[0]

    num = integrate.quad(area, -eps, min(u, eps), epsabs=1e-13, limit=200)[0]
    den = integrate.quad(area, -eps, eps, epsabs=1e-13, limit=200)[0]
    return num / den


def _one_face_2d(u, eps):
    def chord(y1):
        rr = np.sqrt(max(eps * eps - y1 * y1, 0.0))
        return 2 * integrate.quad(lambda y2: _phi(np.hypot(y1, y2), eps), 0, rr, epsabs=1e-14)[0]

    num = integrate.quad(chord, -eps, min(u, eps), epsabs=1e-13, limit=200)[0]
    den = integrate.quad(chord, -eps, eps, epsabs=1e-13, limit=200)[0]
    return num / den


@pytest.mark.parametrize("s", [0, 1, 2, 3, 5, 7])
def test_one_face_values_against_adaptive_quadrature(s):
    eps = 2.5
    # lower face of axis 0 (u = s - eps), axis 1 (and 2) deep inside
    assert cutoff.weight_of((s, 20, 20), (40, 40, 40), eps) == pytest.approx(_one_face_3d(s - eps, eps), abs=1e-9)
    assert cutoff.weight_of((s, 20), (40, 40), eps) == pytest.approx(_one_face_2d(s - eps, eps), abs=1e-9)
    # upper face of the time axis: sample n - s sits s steps from it
    assert cutoff.weight_of((20, 20, 40 - s), (40, 40, 40), eps) == pytest.approx(_one_face_3d(s - eps, eps),
                                                                                  abs=1e-9)


def test_symmetric_values():
    eps = 2.0
    n3 = (30, 30, 30)
    # a sample on the shrunk box's face sees half the bump, on an edge a
    # quarter, at a corner an eighth
    assert cutoff.weight_of((2, 15, 15), n3, eps) == pytest.approx(0.5, abs=1e-10)
    assert cutoff.weight_of((2, 28, 15), n3, eps) == pytest.approx(0.25, abs=1e-10)
    assert cutoff.weight_of((2, 2, 28), n3, eps) == pytest.approx(0.125, abs=1e-10)
    assert cutoff.weight_of((2, 28), (30, 30), eps) == pytest.approx(0.25, abs=1e-10)
    # on the data box's own face and beyond the support: exactly 0 and 1
    assert cutoff.weight_of((0, 15, 15), n3, eps) == 0.0
    assert cutoff.weight_of((4, 4, 26), n3, eps) == 1.0


@pytest.mark.parametrize("d", [2, 3])
def test_reflection_identities(d):
    # y -> -y maps {y1 <= u} onto {y1 >= -u}: W(u) + W(-u) = W(no face), also
    # with a second face present (catches a wrong sign in one box end)
    eps = 2.5
    n = (40,) * d
    mid = (20,) * d
    for s in [1, 2, 3]:
        mirror = int(2 * eps) - s       # u = s - eps  ->  -u
        a = list(mid)
        b = list(mid)
        a[0], b[0] = s, mirror
        assert cutoff.weight_of(tuple(a), n, eps) + cutoff.weight_of(tuple(b), n, eps) == pytest.approx(1.0, abs=1e-10)
        a[1] = b[1] = 1                 # second face on axis 1
        free = list(mid)
        free[1] = 1
        assert cutoff.weight_of(tuple(a), n, eps) + cutoff.weight_of(tuple(b), n, eps) == \
            pytest.approx(cutoff.weight_of(tuple(free), n, eps), abs=1e-10)


def test_monotone_and_bounded_over_a_grid():
    g = dict(n1=12, n2=10, nt=20)
    w = cutoff.weights(g, 2.0)
    assert w.min() >= 0.0 and w.max() <= 1.0
    assert np.all(np.diff(w[:6, 5, 10]) >= 0)       # rising away from the x1 = 0 face
    assert np.all(np.diff(w[5, 5, 10:]) <= 0)       # falling towards the t = nt face
    assert np.all(w[:, :, 0] == 0) and np.all(w[0] == 0)
    # same weights on both ends of an axis at equal distance from the faces
    assert w[1, 5, 10] == pytest.approx(w[11, 5, 10])


def test_printed_mollifier_underflows():
    # the printed exp(-1/(eps - r^2)^4) with eps = (4 steps)^2 at 512 samples
    # per unit: zero in double precision everywhere, so it cannot be the
    # intended bump
    eps_p = (4.0 / 512) ** 2
    r2 = np.linspace(0, eps_p, 1001, endpoint=False)
    with np.errstate(over="ignore"):
        vals = np.exp(-1.0 / (eps_p - r2) ** 4)
    assert np.all(vals == 0.0)
