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
