"""Pins of the oracle's Monte-Carlo QED step (Sec. IV, Method I in optical-
depth form): event statistics, recoil and pair kinematics.  CPU only."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O
from oracle import qed_step as Q

SEED = 2104


def leptons(n, chi, gamma, tau_thr):
    u = math.sqrt(gamma ** 2 - 1)
    return dict(u=[[u] * n, [0.0] * n, [0.0] * n], chi=[chi] * n, tau=[0.0] * n, tau_thr=list(tau_thr),
                id=list(range(1, n + 1)), w=[1.0] * n, pos=list(range(n)))


def test_emission_probability_per_step():
    """With tau_thr = -ln r, the chance that one step of W dt fires is
    1 - exp(-W dt) (the Poisson process of Method I)."""
    n, chi, gamma, hbar_w = 3000, 0.49, 1000.0, 2.4263e-6
    rates = Q.Rates(nodes=256)
    W = Q.A_CONST / hbar_w * rates.frad(chi) / gamma
    dt = 0.3 / W
    thr = [Q.first_threshold(SEED, i + 1, 0) for i in range(n)]
    L = leptons(n, chi, gamma, thr)
    Q.lepton_step(L, SEED, 1, dt, hbar_w, 2.0, rates, None)
    fired = sum(1 for t in L["tau"] if t == 0.0)
    p = 1 - math.exp(-0.3)
    assert abs(fired - n * p) < 4 * math.sqrt(n * p * (1 - p))


def test_recoil_is_collinear_and_conserves_momentum():
    n, chi, gamma, hbar_w = 200, 4.9, 1000.0, 2.4263e-6
    rates = Q.Rates(nodes=256)
    L = leptons(n, chi, gamma, [0.0] * n)  # every lepton fires
    out = []
    Q.lepton_step(L, SEED, 3, 1e-3, hbar_w, 0.0, rates, out)
    assert len(out) == n
    u0 = math.sqrt(gamma ** 2 - 1)
    for p, ph in enumerate(out):
        eps = math.sqrt(sum(c * c for c in ph["k"]))
        assert L["u"][1][p] == 0.0 and L["u"][2][p] == 0.0
        assert L["u"][0][p] == pytest.approx(max(0.0, u0 - eps), rel=1e-12, abs=1e-9)
        assert ph["id"] == Q.child_id(SEED, p + 1, 3, 1)
        assert L["tau"][p] == 0.0 and L["tau_thr"][p] > 0


def test_emitted_spectrum_follows_eq23():
    """The photon energy fractions drawn at chi = 4.9 follow the cumulative
    spectrum of Eq. 23 (KS test against the oracle's quadrature CDF)."""
    n, chi, gamma, hbar_w = 4000, 4.9, 1000.0, 2.4263e-6
    rates = Q.Rates(nodes=256)
    L = leptons(n, chi, gamma, [0.0] * n)
    out = []
    Q.lepton_step(L, SEED, 5, 1e-3, hbar_w, 0.0, rates, out)
    u = np.array([math.sqrt(sum(c * c for c in ph["k"])) / gamma for ph in out])
    F = O.frad(chi)
    cdf = lambda x: np.array([O.compton_cum(chi, float(v)) / F for v in np.atleast_1d(x)])  # noqa: E731
    res = stats.kstest(u, cdf)
    assert res.pvalue > 1e-3


def test_pair_kinematics():
    n, chi, eps, hbar_w = 300, 4.9, 1000.0, 2.4263e-6
    rates = Q.Rates(nodes=256)
    P = dict(k=[[eps] * n, [0.0] * n, [0.0] * n], chi=[chi] * n, tau=[0.0] * n, tau_thr=[0.0] * n,
             id=list(range(10, 10 + n)), w=[1.0] * n, pos=list(range(n)))
    pos, ele = [], []
    Q.photon_decay(P, SEED, 2, 1e-3, hbar_w, rates, pos, ele)
    assert len(pos) == len(ele) == n and all(w == 0.0 for w in P["w"])
    xs = []
    for a, b in zip(pos, ele):
        ea = math.sqrt(1 + sum(c * c for c in a["u"]))
        eb = math.sqrt(1 + sum(c * c for c in b["u"]))
        assert ea + eb == pytest.approx(eps, rel=1e-9)
        assert a["u"][1] == 0.0 and b["u"][2] == 0.0
        xs.append(ea / eps)
    F = O.fpair(chi)
    cdf = lambda x: np.array([O.pair_cum(chi, float(v)) / F for v in np.atleast_1d(x)])  # noqa: E731
    assert stats.kstest(np.array(xs), cdf).pvalue > 1e-3


# ---------------------------------------------------------------- Method II

@pytest.mark.parametrize("chi", [0.05, 0.49, 4.9, 49.0])
def test_method2_mean_acceptance_is_the_total_rate(chi):
    """Averaged over the proposal r1 ~ U(0,1), Method II's acceptance is the
    emission probability W dt of the step (W from the pinned F_rad of Eq. 23);
    a wrong Jacobian, prefactor or time factor breaks the equality."""
    from scipy import integrate
    gamma, hbar_w, dt = 800.0, 2.4263e-6, 0.01
    f = lambda r: Q.emission_acceptance(chi, gamma, r, dt, hbar_w)  # noqa: E731
    mean, _ = integrate.quad(f, 0.0, 1.0, limit=400, epsabs=0.0, epsrel=1e-11)
    W = Q.A_CONST / hbar_w * O.frad(chi) / gamma
    assert mean == pytest.approx(W * dt, rel=1e-7)


@pytest.mark.parametrize("chi", [0.49, 4.9, 49.0])
def test_method2_mean_pair_acceptance_is_the_total_rate(chi):
    from scipy import integrate
    eps, hbar_w, dt = 900.0, 2.4263e-6, 0.01
    f = lambda x: Q.pair_acceptance(chi, eps, x, dt, hbar_w)  # noqa: E731
    mean, _ = integrate.quad(f, 0.0, 1.0, points=[0.5], limit=400, epsabs=0.0, epsrel=1e-11)
    W = Q.A_CONST / hbar_w * O.fpair(chi) / eps
    assert mean == pytest.approx(W * dt, rel=1e-7)


def test_method2_emission_count_and_spectrum():
    """One Method II step with W dt = 0.25 fires in a quarter of the leptons
    (binomial, 4 sigma) and the photon energies follow the cumulative spectrum
    of Eq. 23 (KS); every photon has u0 = r1^3 of its lepton's stream."""
    n, chi, gamma, hbar_w = 4000, 4.9, 1000.0, 2.4263e-6
    W = Q.A_CONST / hbar_w * O.frad(chi) / gamma
    dt = 0.25 / W
    L = leptons(n, chi, gamma, [1.0] * n)
    out = []
    sat = Q.lepton_step_method2(L, SEED, 7, dt, hbar_w, 0.0, out)
    assert not sat
    assert abs(len(out) - 0.25 * n) < 4 * math.sqrt(n * 0.25 * 0.75)
    u = []
    for ph in out:
        pid = ph["pos"] + 1
        r1, _ = O.qed_uniforms(SEED, pid, 7, 0)
        e = math.sqrt(sum(c * c for c in ph["k"]))
        assert e == pytest.approx(r1 ** 3 * gamma, rel=1e-12)
        u.append(e / gamma)
    assert all(t == 0.0 for t in L["tau"])  # Method II leaves tau alone
    F = O.frad(chi)
    cdf = lambda x: np.array([O.compton_cum(chi, float(v)) / F for v in np.atleast_1d(x)])  # noqa: E731
    assert stats.kstest(np.array(u), cdf).pvalue > 1e-3


def test_method2_pair_count_and_spectrum():
    n, chi, eps, hbar_w = 3000, 4.9, 1000.0, 2.4263e-6
    W = Q.A_CONST / hbar_w * O.fpair(chi) / eps
    dt = 0.25 / W
    P = dict(k=[[eps] * n, [0.0] * n, [0.0] * n], chi=[chi] * n, tau=[0.0] * n, tau_thr=[1.0] * n,
             id=list(range(10, 10 + n)), w=[1.0] * n, pos=list(range(n)))
    pos, ele = [], []
    assert not Q.photon_decay_method2(P, SEED, 4, dt, hbar_w, pos, ele)
    assert len(pos) == len(ele)
    assert abs(len(pos) - 0.25 * n) < 4 * math.sqrt(n * 0.25 * 0.75)
    assert sum(1 for w in P["w"] if w == 0.0) == len(pos)
    xs = [math.sqrt(1 + sum(c * c for c in a["u"])) / eps for a in pos]
    F = O.fpair(chi)
    cdf = lambda x: np.array([O.pair_cum(chi, float(v)) / F for v in np.atleast_1d(x)])  # noqa: E731
    assert stats.kstest(np.array(xs), cdf).pvalue > 1e-3


def test_method2_reports_saturation():
    """An acceptance above 1 means the step is too long for the rate."""
    n, chi, gamma, hbar_w = 50, 4.9, 1000.0, 2.4263e-6
    W = Q.A_CONST / hbar_w * O.frad(chi) / gamma
    assert not Q.lepton_step_method2(leptons(n, chi, gamma, [1.0] * n), SEED, 1, 0.1 / W, hbar_w, 0.0, None)
    assert Q.lepton_step_method2(leptons(n, chi, gamma, [1.0] * n), SEED, 1, 5.0 / W, hbar_w, 0.0, None)


# ------------------------------------------------ photon move and chi_gamma

def _linear_plane(g, comp, a, b):
    """Plane of component `comp` whose value at its own staggered node is
    a + b x (x the node's absolute x coordinate)."""
    sx = {0: 0.5, 1: 0.0, 2: 0.0, 3: 0.0, 4: 0.5, 5: 0.5}[comp]
    n = list(g.n) + [1] * (3 - len(g.n))
    x = (np.arange(n[0]) + sx) * g.d[0]
    return np.broadcast_to(a + b * x, g.shape).copy()


@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (3, 2), (2, 4), (3, 4)])
def test_photon_chi_in_a_linear_field(dim, order):
    """A photon moving in the x-y plane across B_z = b0 + b1 x (E = 0) has
    chi_gamma = (hbar w) eps |B_z| at its new position x + dt k_x / eps: the
    gather of a linear field is exact on each component's own stagger, so a
    wrong move, stagger or chi formula shows."""
    n = (24, 16) if dim == 2 else (24, 12, 10)
    d = (0.3, 0.25, 0.2)[:dim]
    g = O.Grid(dim, n, d, 0.1, order)
    F = [np.zeros(g.shape) for _ in range(6)]
    b0, b1 = 0.7, 0.31
    F[5] = _linear_plane(g, 5, b0, b1)
    rng = np.random.default_rng(4)
    m, hbar_w = 40, 1e-3
    th = rng.uniform(0, 2 * np.pi, m)
    eps = rng.uniform(3.0, 50.0, m)
    x0 = [rng.uniform(6 * d[0], (n[0] - 6) * d[0], m)] + [rng.uniform(0, n[a] * d[a], m) for a in range(1, dim)]
    ph = dict(x=[list(v) for v in x0], k=[list(eps * np.cos(th)), list(eps * np.sin(th)), [0.0] * m],
              w=[1.0] * m)
    Q.photon_move_chi(g, F, ph, g.dt, hbar_w)
    xn = x0[0] + g.dt * np.cos(th)
    assert np.allclose(ph["x"][0], xn, rtol=0, atol=1e-12)
    yn = (x0[1] + g.dt * np.sin(th)) % (n[1] * d[1])
    assert np.allclose(ph["x"][1], yn, rtol=0, atol=1e-12)
    assert np.allclose(ph["chi"], hbar_w * eps * (b0 + b1 * xn), rtol=1e-12)


def test_photon_chi_of_plane_waves():
    """Against a plane wave E_y = B_z = a along x, a photon moving with the
    wave has chi_gamma = 0 and one moving against it 2 (hbar w) eps a."""
    g = O.Grid(2, (20, 12), (0.2, 0.2), 0.1, 2)
    F = [np.zeros(g.shape) for _ in range(6)]
    a = 0.9
    F[1][...] = a
    F[5][...] = a
    m = 6
    eps = np.linspace(5.0, 30.0, m)
    for sign, want in ((1.0, 0.0), (-1.0, 2.0)):
        ph = dict(x=[[1.0] * m, [1.0] * m], k=[list(sign * eps), [0.0] * m, [0.0] * m], w=[1.0] * m)
        Q.photon_move_chi(g, F, ph, g.dt, 1e-3)
        assert np.allclose(ph["chi"], want * 1e-3 * eps * a, rtol=1e-12, atol=1e-15)


def test_photon_absorbed_at_x_faces():
    """With absorbing x faces a photon whose new x leaves [0, (n-1) dx] gets
    w = 0 and chi = 0; the rest keep their weight; y wraps."""
    n, d, dt = (16, 8), (0.2, 0.2), 0.1
    g = O.Grid(2, n, d, dt, 2, absorb_x=1)
    F = [np.full(g.shape, 0.3) for _ in range(6)]
    xs = [0.05, 0.05, 2.0, (n[0] - 1) * d[0] - 0.05, (n[0] - 1) * d[0] - 0.05, 1.0]
    kx = [-1.0, 1.0, -1.0, 1.0, -1.0, 0.0]
    ky = [0.0, 0.0, 0.0, 0.0, 0.0, 1.0]
    ph = dict(x=[list(xs), [0.5, 0.5, 0.5, 0.5, 0.5, n[1] * d[1] - 0.01]], k=[kx, ky, [0.0] * 6], w=[1.0] * 6)
    Q.photon_move_chi(g, F, ph, dt, 1e-3)
    assert ph["w"] == [0.0, 1.0, 1.0, 0.0, 1.0, 1.0]
    assert ph["chi"][0] == 0.0 and ph["chi"][3] == 0.0 and ph["chi"][1] > 0.0
    assert abs(ph["x"][1][5] - (0.09)) < 1e-12


def test_cascade_bookkeeping():
    """The oracle's Fig. 9 cascade run: every pair adds one positron and
    one electron and removes its photon; the field does no work; pair
    members carry the photon's energy (a member whose share x eps is below
    m c^2 is left at rest, so a pair may add up to 2 m c^2) and an emission's
    recoil loses up to one m c^2 beyond the photon's energy: the total energy
    stays within [start - emissions, start + 2 pairs]."""
    hb = 2.4263e-6
    b0 = 0.009 / hb
    n = 60
    el, po, ph, sat = Q.cascade_uniform_b(b0, 1000.0, n, 12, 0.02, hb, SEED)
    assert not sat
    decayed = sum(1 for w in ph["w"] if w == 0.0)
    assert len(po["w"]) == decayed and len(el["w"]) == n + decayed
    assert decayed > 0 and len(ph["w"]) > 3 * n
    gam = lambda L: sum(math.sqrt(1 + sum(L["u"][a][p] ** 2 for a in range(3))) for p in range(len(L["w"])))  # noqa
    eps = sum(math.sqrt(sum(ph["k"][a][p] ** 2 for a in range(3))) for p in range(len(ph["w"])) if ph["w"][p] != 0)
    total, start = gam(el) + gam(po) + eps, n * 1000.0
    assert start - len(ph["w"]) <= total <= start + 2 * decayed + 1e-9 * start


def test_cascade_electrons_gyrate_between_emissions():
    """Between emissions the uniform magnetic field turns u without changing
    |u| (Boris), by the angle 2 atan(Omega dt / 2) per step."""
    hb = 2.4263e-6
    b0 = 0.001 / hb
    el, _, ph, _ = Q.cascade_uniform_b(b0, 1000.0, 40, 1, 0.1, hb, SEED)
    emitted = {Q.child_id(SEED, i, 0, 1) for i in range(1, 41)} & set(ph["id"])
    quiet = [p for p in range(40) if Q.child_id(SEED, p + 1, 0, 1) not in emitted]
    assert quiet
    u0 = math.sqrt(1000.0 ** 2 - 1)
    for p in quiet:
        u = [el["u"][a][p] for a in range(3)]
        assert math.sqrt(sum(c * c for c in u)) == pytest.approx(u0, rel=1e-14)
        ang = math.atan2(u[1], u[0])
        assert abs(ang) == pytest.approx(2 * math.atan(b0 / 1000.0 * 0.1 / 2), rel=1e-12)
