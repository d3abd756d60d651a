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
