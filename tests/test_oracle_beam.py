"""Pins of the oracle's bunch self-fields (Sec. III(c): rest-frame Poisson
solution, Lorentz-transformed to the lab) against closed forms and Gauss's
law.  CPU only."""
import math

import numpy as np
import pytest
from scipy import special

from oracle import beam as BM

pytestmark = pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")


@pytest.mark.parametrize("r_over_sigma", [0.3, 1.0, 3.0])
def test_sphere_at_rest(r_over_sigma):
    """A spherical Gaussian charge at rest: by Gauss's law on a sphere,
    E_r = Q/(4 pi r^2) [erf(r / (sqrt2 sigma)) - sqrt(2/pi) (r/sigma)
    exp(-r^2 / (2 sigma^2))], radial."""
    Q, s = 2.0, 0.7
    r = r_over_sigma * s
    n = np.array([0.3, -0.5, 0.81])
    n /= np.linalg.norm(n)
    E = np.array(BM.rest_frame_field(Q, (s, s, s), r * n))
    exact = Q / (4 * math.pi * r * r) * (special.erf(r / (math.sqrt(2) * s)) -
                                         math.sqrt(2 / math.pi) * (r / s) * math.exp(-r * r / (2 * s * s)))
    assert np.dot(E, n) == pytest.approx(exact, rel=1e-10)
    assert np.linalg.norm(E - np.dot(E, n) * n) < 1e-10 * abs(exact)


@pytest.mark.parametrize("r_over_sigma", [0.3, 1.0, 3.0])
def test_disc_at_rest(r_over_sigma):
    """2D: a circular Gaussian line charge, E_r = Q/(2 pi r) (1 - exp(-r^2 /
    (2 sigma^2)))."""
    Q, s = 2.0, 0.7
    r = r_over_sigma * s
    n = np.array([0.6, -0.8])
    E = np.array(BM.rest_frame_field(Q, (s, s), r * n))
    exact = Q / (2 * math.pi * r) * (1 - math.exp(-r * r / (2 * s * s)))
    assert np.dot(E, n) == pytest.approx(exact, rel=1e-10)
    assert abs(E[0] * n[1] - E[1] * n[0]) < 1e-10 * abs(exact)


def test_far_field_of_an_anisotropic_bunch_is_a_point_charge():
    """Far away (|p| = 170 sigma) the field of an anisotropic bunch is
    Q p / (4 pi |p|^3) up to its quadrupole, of relative size (sigma/|p|)^2."""
    Q, sig = 2.0, (1.5, 0.5, 0.8)
    p = np.array([120.0, -90.0, 70.0])
    E = np.array(BM.rest_frame_field(Q, sig, p))
    R = np.linalg.norm(p)
    assert np.max(np.abs(E / (Q * p / (4 * math.pi * R ** 3)) - 1)) < 5e-4


@pytest.mark.parametrize("dim,gamma", [(3, 3.0), (2, 4.0)])
def test_lab_fields_obey_gauss_law(dim, gamma):
    """In the lab the moving bunch's E has div E = rho_lab (central
    differences, step 1e-3): this ties the x' = gamma x contraction, the
    gamma on E_perp and the gamma sigma_x rest length together."""
    if dim == 3:
        b = BM.Bunch(-1.0, 4.0, (0.0, 0.0, 0.0), (0.5, 0.4, 0.6), gamma)
        pts = [(0.1, 0.2, -0.3), (0.4, -0.5, 0.1)]
    else:
        b = BM.Bunch(1.0, 2.0, (0.0, 0.0), (0.5, 0.3), gamma, dim=2)
        pts = [(0.1, 0.2, 0.0), (0.4, -0.5, 0.0)]
    h = 1e-3
    for pt in pts:
        dv = 0.0
        for a in range(dim):
            pp, pm = list(pt), list(pt)
            pp[a] += h
            pm[a] -= h
            dv += (BM.lab_field(b, a, *pp) - BM.lab_field(b, a, *pm)) / (2 * h)
        rho = BM.lab_density(b, *pt)
        assert dv == pytest.approx(rho, rel=1e-5)


def test_ultrarelativistic_limit_is_the_line_charge_field():
    """As gamma grows the lab field tends to that of the line charge
    Lambda(x) = q n_b 2 pi sigma_r^2 exp(-x^2 / (2 sigma_x^2)) with its
    Gaussian profile, E_r = Lambda (1 - exp(-r^2/(2 sigma_r^2))) / (2 pi r),
    E_x -> 0: the departure shrinks like ln(gamma) / gamma^2 (a slender body's
    correction), and B_z = beta E_y."""
    x, y, z = 0.2, 0.4, -0.3
    r = math.hypot(y, z)
    lam = -4.0 * math.exp(-x * x / (2 * 0.25)) * 2 * math.pi * 0.25
    er = lam * (1 - math.exp(-r * r / 0.5)) / (2 * math.pi * r)
    dep = {}
    for g in (8.0, 16.0, 50.0):
        b = BM.Bunch(-1.0, 4.0, (0.0, 0.0, 0.0), (0.5, 0.5, 0.5), g)
        ey = BM.lab_field(b, 1, x, y, z)
        ex = BM.lab_field(b, 0, x, y, z)
        dep[g] = abs(ey / (er * y / r) - 1)
        assert abs(ex / ey) < 2 * (1 + math.log(g)) / g ** 2
        assert 0.5 * math.log(g) / g ** 2 < dep[g] < 2 * (1 + math.log(g)) / g ** 2
        beta = math.sqrt(1 - 1 / g ** 2)
        assert BM.lab_field(b, 5, x, y, z) == pytest.approx(beta * ey, rel=1e-12)
    assert dep[50.0] < dep[16.0] < dep[8.0]
