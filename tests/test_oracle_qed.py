"""Pins of the oracle's QED module (Sec. IV, Eqs. 23-24) and of its surrogate
network reference.  CPU only: SciPy's Bessel routines and adaptive quadrature
are an independent route; the classical and asymptotic limits are closed forms."""
import math
import os

import numpy as np
import pytest
from scipy import integrate, special

import oracle as O
from oracle import mlp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALPHA = 1.0 / 137.035999084


@pytest.mark.parametrize("nu", [1 / 3, 2 / 3])
def test_bessel_k_matches_library(nu):
    for y in [1e-8, 1e-4, 0.01, 0.3, 1.0, 4.0, 20.0, 150.0, 600.0]:
        assert O.bessel_k(nu, y) == pytest.approx(special.kv(nu, y), rel=1e-12)


def test_int_k13_matches_library():
    for y in [1e-6, 1e-3, 0.2, 1.0, 3.0, 12.0, 60.0]:
        ref = integrate.quad(lambda s: special.kv(1 / 3, s), y, np.inf, epsabs=0, epsrel=1e-13,
                             limit=500)[0]
        assert O.int_k13(y) == pytest.approx(ref, rel=1e-11)
    # int_0^inf K_{1/3} = pi / sqrt(3)
    assert O.int_k13(1e-12) == pytest.approx(math.pi / math.sqrt(3), rel=1e-6)


def scipy_frad(chi):
    def f(u):
        y = 2 * u / (3 * (1 - u) * chi)
        if y > 700:
            return 0.0
        ik = integrate.quad(lambda s: special.kv(1 / 3, s), y, np.inf, epsrel=1e-13, limit=200)[0]
        return (u * u - 2 * u + 2) / (1 - u) * special.kv(2 / 3, y) - ik
    # u = s^3 substitution, independent quadrature (QUADPACK)
    return integrate.quad(lambda s: 3 * s * s * f(s ** 3), 0, 1, epsrel=1e-11, limit=400)[0]


def scipy_fpair(chi):
    def f(x):
        y = 2 / (3 * chi * x * (1 - x))
        if y > 700:
            return 0.0
        ik = integrate.quad(lambda s: special.kv(1 / 3, s), y, np.inf, epsrel=1e-13, limit=200)[0]
        return (x * x + (1 - x) ** 2) / (x * (1 - x)) * special.kv(2 / 3, y) + ik
    return 2 * integrate.quad(f, 0, 0.5, epsrel=1e-11, limit=400)[0]


@pytest.mark.parametrize("chi", [1e-3, 0.49, 4.9, 49.0])
def test_frad_matches_library_quadrature(chi):
    assert O.frad(chi) == pytest.approx(scipy_frad(chi), rel=1e-8)


@pytest.mark.parametrize("chi", [0.2, 0.49, 4.9, 49.0])
def test_fpair_matches_library_quadrature(chi):
    assert O.fpair(chi) == pytest.approx(scipy_fpair(chi), rel=1e-8)


@pytest.mark.parametrize("chi", [1e-10, 1e-8, 2e-9, 1e-6])
def test_frad_classical_limit_at_tiny_chi(chi):
    """Far below the tables: F_rad = (5 pi / 2) chi (1 - c chi + ...); the
    quadrature must find the spectrum at u ~ chi."""
    assert O.frad(chi) / (2.5 * math.pi * chi) == pytest.approx(1.0, abs=2 * chi + 1e-9)


def test_frad_classical_limit():
    """chi -> 0: W_rad -> (5/(2 sqrt 3)) alpha (m c^2/hbar) chi / gamma, i.e.
    F_rad / (5 pi chi / 2) -> 1 (with corrections of order chi)."""
    r = [O.frad(c) / (2.5 * math.pi * c) for c in (1e-4, 1e-3)]
    assert r[0] == pytest.approx(1.0, abs=2e-3)
    assert abs(r[0] - 1) < abs(r[1] - 1)


def test_radiated_power_larmor_limit():
    """chi -> 0: the emitted power int u dW/du du tends to the classical
    (Larmor) value (2/3) alpha chi^2 m c^2 (m c^2/hbar), i.e.
    int u * bracket du -> 2 pi chi^2 / sqrt(3)."""
    chi = 1e-3
    val = integrate.quad(lambda s: 3 * s * s * s ** 3 * O.compton_bracket(s ** 3, chi), 0, 1,
                         epsrel=1e-10, limit=400, points=[0.05, 0.1, 0.2])[0]
    assert val / (2 * math.pi * chi * chi / math.sqrt(3)) == pytest.approx(1.0, abs=1e-2)


def test_fpair_small_chi_asymptote():
    """chi -> 0: W_pair -> (3 sqrt3 / (16 sqrt2)) alpha (m c^2/hbar) chi
    exp(-8/(3 chi)) / eps_gamma (Erber), i.e. F_pair -> sqrt3 pi chi (3/16)
    sqrt(3/2) exp(-8/(3 chi))."""
    chi = 0.02
    ref = math.sqrt(3) * math.pi * chi * 3 / 16 * math.sqrt(1.5) * math.exp(-8 / (3 * chi))
    assert O.fpair(chi) / ref == pytest.approx(1.0, abs=0.02)


def test_pair_spectrum_symmetric():
    for chi in (0.3, 5.0):
        for x in (0.01, 0.1, 0.3, 0.45):
            assert O.pair_bracket(x, chi) == pytest.approx(O.pair_bracket(1 - x, chi), rel=1e-13)


def test_frad_large_chi_power_law():
    """chi >> 1: F_rad grows like chi^(2/3) (the oracle's range ends at chi = 1e3)."""
    a, b = O.frad(1e2), O.frad(1e3)
    assert math.log(b / a) / math.log(10) == pytest.approx(2 / 3, abs=0.04)


@pytest.mark.parametrize("chi", [0.05, 0.49, 4.9, 49.0])
def test_compton_inverse_cdf(chi):
    F = O.frad(chi)
    prev = 0.0
    for r in (0.01, 0.2, 0.5, 0.8, 0.99):
        u = O.compton_inverse(chi, r)
        assert O.compton_cum(chi, u) / F == pytest.approx(r, abs=1e-9)
        assert prev < u < 1
        prev = u


@pytest.mark.parametrize("chi", [0.49, 4.9])
def test_pair_inverse_cdf(chi):
    F = O.fpair(chi)
    for r in (0.05, 0.5, 0.95):
        x = O.pair_inverse(chi, r)
        assert O.pair_cum(chi, x) / F == pytest.approx(r, abs=1e-9)
    assert O.pair_inverse(chi, 0.5) == pytest.approx(0.5, abs=1e-9)


def test_compton_mean_photon_energy_fraction_vs_library():
    """<u> = int u dW / int dW, the first moment of the Fig. 8(a-c) spectra,
    computed with SciPy's routines as an independent route."""
    chi = 4.9
    num = integrate.quad(lambda s: 3 * s ** 5 * O.compton_bracket(s ** 3, chi), 0, 1,
                         epsrel=1e-11, limit=400)[0]
    mean = num / O.frad(chi)

    def f(u):
        y = 2 * u / (3 * (1 - u) * chi)
        if y > 700:
            return 0.0
        ik = integrate.quad(lambda s: special.kv(1 / 3, s), y, np.inf, epsrel=1e-13)[0]
        return (u * u - 2 * u + 2) / (1 - u) * special.kv(2 / 3, y) - ik
    ref = integrate.quad(lambda s: 3 * s ** 5 * f(s ** 3), 0, 1, epsrel=1e-11, limit=400)[0]
    assert mean == pytest.approx(ref / scipy_frad(chi), rel=1e-8)


def test_chi_of_particle():
    """chi_e = (hbar w / m c^2) |F_mu_nu p^nu|: in a pure magnetic field
    perpendicular to u it is (hbar w/mc^2) |u| B; for E parallel to u it is
    (hbar w/mc^2) |E| (a longitudinal field is unchanged by the boost)."""
    h = 2.4263e-6
    u = np.array([100.0, 0, 0])
    g = math.sqrt(1 + u @ u)
    assert O.chi(h, g, u, np.zeros(3), np.array([0, 0, 30.0])) == pytest.approx(h * 100 * 30)
    assert O.chi(h, g, u, np.array([5.0, 0, 0]), np.zeros(3)) == pytest.approx(h * 5.0, rel=1e-9)
    # counter-propagating plane wave E_y = B_z = a: chi = h a (gamma + u_x)... for u along -x
    a = 7.0
    u = np.array([-50.0, 0, 0])
    g = math.sqrt(1 + u @ u)
    assert O.chi(h, g, u, np.array([0, a, 0]), np.array([0, 0, a])) == pytest.approx(
        h * a * (g + 50.0), rel=1e-12)


def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        assert O.philox4x32_10(v[0:4], v[4:6]) == v[6:10]


def test_uniforms_in_open_interval():
    assert 0 < O.u01(0, 0) < 1e-15
    assert 1 - 1e-15 < O.u01(0xFFFFFFFF, 0xFFFFFFFF) < 1
    xs = [O.qed_uniforms(642, p, 3, 0) for p in range(2000)]
    a = np.array(xs)
    assert np.all((a > 0) & (a < 1))
    assert abs(a.mean() - 0.5) < 0.02


def test_mlp_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = mlp.init_params(rng)
    for k in p:
        p[k] = p[k] + 0.1 * rng.standard_normal(p[k].shape)
    X = rng.uniform(-1, 1, (16, 4))
    T = rng.uniform(-1, 1, (16, 2))
    g = mlp.backward(p, X, T)
    eps = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp = mlp.loss(p, X, T)
            flat[idx] = old - eps
            lm = mlp.loss(p, X, T)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            assert g[k].reshape(-1)[idx] == pytest.approx(fd, rel=1e-6, abs=1e-10)
