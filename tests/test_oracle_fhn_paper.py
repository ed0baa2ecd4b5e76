"""Pins of the oracle's model of the paper's modified FH-N network (Sec. 5.1
eqs. eqUd, eqVd, eqStimulusRegion-eqPsi_ijt; constants of Sec. 5.2); CPU
only.  Each pin comes from outside the oracle's own formula:
  - the node's fixed point (U*, V*), from numpy's roots of the cubic that
    eliminating V from the two nullclines leaves, stays put under a
    noise-free step without coupling, and so do the roots 0, +-sqrt(3.6) of
    p3 with V = 0 (a wrong sign of the cubic moves them);
  - the neighbour sets of Sec. 5.2 (2 at a corner, 3 on a side, 4 inside)
    from an impulse field;
  - the stimulus region on hand-built fields (open band, node or neighbour);
  - the event centre is uniform over the region (chi-square), the event
    rate is eps (binomial), an event stimulates its centre and neighbours
    with F~ for exactly l0 steps and overlapping events do not add;
  - the forcing pulse hits the 2 x 2 corner for `width` steps per period;
  - the noise is sigma~ sqrt(h) on U only (chi-square of the variance).
"""
import numpy as np
import pytest
from scipy import stats

import pf_inputs

J = 32
NN = J * J


def _spec(**kw):
    s = pf_inputs.fhn_paper(J)
    ext = list(s["params_ext"])
    par = list(s["params"])
    sd = list(s["noise_sd"])
    for k, v in kw.items():
        if k == "a2": par[0] = v
        elif k == "c": par[1] = v
        elif k == "b0": par[2] = v
        elif k == "b1": par[3] = v
        elif k == "b2": ext[0] = v
        elif k == "amp": ext[1] = v
        elif k == "eps": ext[2] = v
        elif k == "width": ext[7] = v
        elif k == "sd": sd = [v, 0.0]
    s.update(params=tuple(par), params_ext=tuple(ext), noise_sd=tuple(sd))
    return s


def _state(U, V=None, ring=None):
    x = np.full(2 * NN + 28, -1.0)
    x[:NN] = U
    x[NN:2 * NN] = 0.0 if V is None else V
    if ring is not None:
        x[2 * NN:2 * NN + len(ring)] = ring
    return x


def test_rest_point_and_cubic_roots(orc):
    # no coupling, no noise, no stimuli, no forcing
    m = orc.Model(_spec(c=0.0, sd=0.0, eps=0.0, width=0.0))
    a2, b0, b1, b2 = 3.6, 2.1, -0.6, 0.6
    # V* = -(b0 U + b2) / b1 on the V-nullcline; a2 U - U^3 - V* = 0
    roots = np.roots([-1.0, 0.0, a2 + b0 / b1, b2 / b1])
    us = roots[np.isreal(roots)].real
    assert us.size == 1
    u = us[0]
    v = -(b0 * u + b2) / b1
    assert u == pytest.approx(-1.0332, abs=1e-3)
    xo, ev = orc.fhnp_step(m, 1, 2, 0, 0, 7, _state(np.full(NN, u), np.full(NN, v)))
    assert ev == -1
    assert np.allclose(xo[:NN], u, atol=1e-12) and np.allclose(xo[NN:2 * NN], v, atol=1e-12)
    # roots of p3 with V = 0 (and no recovery, so that V stays 0)
    m0 = orc.Model(_spec(c=0.0, sd=0.0, eps=0.0, width=0.0, b0=0.0, b1=0.0, b2=0.0))
    for r in (0.0, np.sqrt(3.6), -np.sqrt(3.6)):
        xo, _ = orc.fhnp_step(m0, 1, 2, 0, 0, 3, _state(np.full(NN, r)))
        assert np.allclose(xo[:NN], r, atol=1e-12)
    # away from the roots the cubic pulls back towards +-sqrt(3.6) (stable
    # outer branches): the printed positive leading coefficient would push out
    xo, _ = orc.fhnp_step(m0, 1, 2, 0, 0, 3, _state(np.full(NN, 2.5)))
    assert np.all(xo[:NN] < 2.5)


def test_neighbour_sets(orc):
    # impulse of 1 at one node, everything else 0: with a2 = 0 (p3 = -u^3),
    # coupling c = 1, the neighbours move by h and the rest stays at 0
    m = orc.Model(_spec(a2=0.0, c=1.0, sd=0.0, eps=0.0, width=0.0, b0=0.0, b1=0.0, b2=0.0))
    h = 5e-3
    for (i, j), want in (((0, 0), 2), ((0, J - 1), 2), ((J - 1, 0), 2), ((J - 1, J - 1), 2),
                         ((0, 5), 3), ((7, 0), 3), ((J - 1, 9), 3), ((4, J - 1), 3),
                         ((10, 11), 4)):
        U = np.zeros(NN)
        U[i * J + j] = 1.0
        xo, _ = orc.fhnp_step(m, 1, 2, 0, 0, 3, _state(U))
        d = xo[:NN].copy()
        d[i * J + j] = 0.0
        moved = np.flatnonzero(d)
        assert moved.size == want
        assert np.allclose(d[moved], h)
        for k in moved:
            assert abs(k // J - i) + abs(k % J - j) == 1


def test_stimulus_region(orc):
    m = orc.Model(_spec())
    U = np.zeros(NN)
    U[10 * J + 10] = -1.7
    c, reg = orc.fhnp_region(m, U)
    assert c == 5 and set(np.flatnonzero(reg)) == {330, 330 - J, 330 + J, 329, 331}
    U[0] = -1.75
    c, reg = orc.fhnp_region(m, U)
    assert c == 8 and reg[0] and reg[1] and reg[J]
    # the band is open: the thresholds themselves are outside
    U = np.zeros(NN)
    U[100], U[500] = -1.8, -1.6
    assert orc.fhnp_region(m, U)[0] == 0


def test_event_centre_uniform_and_rate(orc):
    m = orc.Model(_spec(eps=1.0, sd=0.0))
    U = np.zeros(NN)
    U[10 * J + 10] = -1.7
    region = [330, 330 - J, 330 + J, 329, 331]
    R = 5000
    cnt = {k: 0 for k in region}
    for n in range(R):
        _, ev = orc.fhnp_step(m, 4, 2, 0, 0, n, _state(U))
        assert ev in cnt
        cnt[ev] += 1
    obs = np.array(list(cnt.values()))
    assert stats.chisquare(obs).pvalue > 1e-4
    # Bernoulli rate eps
    m3 = orc.Model(_spec(eps=0.3, sd=0.0))
    ev = np.array([orc.fhnp_step(m3, 5, 2, 1, 0, n, _state(U))[1] >= 0 for n in range(20000)])
    assert abs(ev.mean() - 0.3) < 5 * np.sqrt(0.3 * 0.7 / ev.size)
    # nothing happens where the region is empty
    assert all(orc.fhnp_step(m, 4, 2, 0, 0, n, _state(np.zeros(NN)))[1] == -1 for n in range(50))


def test_stimulus_duration_and_overlap(orc):
    # no dynamics but the stimulus: an event at step 3 centred on node 330
    # puts F~ h on the centre and its 4 neighbours at steps 3 .. 3 + l0 - 1
    m = orc.Model(_spec(a2=0.0, c=0.0, sd=0.0, eps=0.0, width=0.0, b0=0.0, b1=0.0, b2=0.0))
    amp, h, l0 = 200.0, 5e-3, 25
    ring = [-1.0] * 25
    ring[3] = 330.0              # the event of step 3, in ring slot 3
    group = [330, 330 - J, 330 + J, 329, 331]
    for n in range(4, 3 + l0 + 3):
        # (step 3 + l0 writes its own event, here none, into slot 3); the
        # ring is carried from step to step, U and V restart from 0
        xo, _ = orc.fhnp_step(m, 1, 2, 0, 0, n, _state(np.zeros(NN), ring=ring))
        ring = list(xo[2 * NN:2 * NN + 25])
        on = n < 3 + l0
        for k in group:
            assert xo[k] == pytest.approx(amp * h if on else 0.0, abs=1e-12), (n, k)
        assert np.count_nonzero(xo[:NN]) == (5 if on else 0)
    # two overlapping events: the shared node still gets F~ once
    r = [-1.0] * 25
    r[0], r[1] = 330.0, 331.0
    xo, _ = orc.fhnp_step(m, 1, 2, 0, 0, 2, _state(np.zeros(NN), ring=r))
    assert xo[330] == pytest.approx(amp * h) and xo[331] == pytest.approx(amp * h)


def test_forcing_schedule(orc):
    m = orc.Model(_spec(a2=0.0, c=0.0, sd=0.0, eps=0.0, b0=0.0, b1=0.0, b2=0.0))
    amp, h = 200.0, 5e-3
    corner = [0, 1, J, J + 1]
    for n, on in ((0, True), (24, True), (25, False), (3999, False), (4000, True), (4024, True),
                  (4025, False)):
        xo, _ = orc.fhnp_step(m, 1, 2, 0, 0, n, _state(np.zeros(NN)))
        assert np.allclose(xo[corner], amp * h if on else 0.0, atol=1e-12), n
        rest = np.delete(xo[:NN], corner)
        assert np.all(rest == 0.0)


def test_noise_on_u_only(orc):
    m = orc.Model(_spec(a2=0.0, c=0.0, eps=0.0, width=0.0, b0=0.0, b1=0.0, b2=0.0))
    h, var = 5e-3, 0.5
    zs = []
    for n in range(20):
        xo, _ = orc.fhnp_step(m, 9, 2, 3, 1, n, _state(np.zeros(NN)))
        assert np.all(xo[NN:2 * NN] == 0.0)
        zs.append(xo[:NN])
    z = np.concatenate(zs)
    dof = z.size - 1
    s2 = np.var(z, ddof=1)
    lo, hi = stats.chi2.ppf([1e-5, 1 - 1e-5], dof)
    assert lo * var * h / dof < s2 < hi * var * h / dof
