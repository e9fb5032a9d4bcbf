"""The spring state as the GPU law stores it, checked against the oracle's law
(Section 2.1, the modified Ramberg-Osgood skeleton with Masing branches).

The oracle keeps the largest strain reached on the skeleton, gamma_m.  The
GPU law keeps s_m = S(gamma_m / gamma_ref) / (G0 gamma_ref) instead: the
skeleton e = s (1 + (2 s)^beta) gives gamma_m back explicitly, the damping
1 - S(e_m)/e_m becomes p_m / (1 + p_m) with p_m = (2 s_m)^beta, and a reversal
on the skeleton takes the stress +-G0 gamma_ref s_m.  This test re-states that
update in plain Python (the update rules only; skeleton inversions through the
oracle's own routine) and runs it beside the oracle along random strain paths
that reverse on the skeleton and on branches, rejoin the skeleton and close
inner loops: stresses, tangents, damping and the on-skeleton flag agree to
rounding.  It pins the state form; the GPU kernel itself is held to the oracle
by the parity tests."""
import ctypes as C
import math

import numpy as np
import pytest

import oracle


def _pow2s(s, beta):
    return (2.0 * s) ** beta


class SmSpring:
    """One spring in the stored form of the GPU law (the update's rules in
    the order the kernel applies them)."""

    def __init__(self, depth):
        self.gp = self.gr = self.tr = self.sm = 0.0
        self.dir, self.skel = 0, 1
        self.od = []  # older branch origins (gr, tr), oldest first
        self.depth = depth

    def step(self, dg, G0, gref, beta, hmax):
        S = lambda e: oracle.ro_inverse(e, beta)
        dsg = 1 if dg > 0 else (-1 if dg < 0 else 0)
        reverse = dsg != 0 and self.dir != 0 and dsg != self.dir
        pm, gm = 0.0, abs(self.gp)
        if (not self.skel or reverse) and self.sm > 0:
            pm = _pow2s(self.sm, beta)
            if not self.skel:
                gm = gref * self.sm * (1.0 + pm)
        if dsg != 0:
            if reverse:
                if self.skel:
                    trev = G0 * gref * math.copysign(self.sm, self.gp)
                else:
                    trev = self.tr + 2.0 * G0 * gref * S(0.5 * (self.gp - self.gr) / gref)
                    if self.depth > 1:
                        if len(self.od) == self.depth - 1:
                            self.od.pop(0)
                        self.od.append((self.gr, self.tr))
                self.tr, self.gr, self.skel = trev, self.gp, 0
            self.dir = dsg
            g = self.gp + dg
            if not self.skel and dsg * g >= gm:
                self.skel, self.od = 1, []
            while self.depth > 1 and not self.skel and len(self.od) >= 2 and dsg * g >= dsg * self.od[-1][0]:
                self.gr, self.tr = self.od[-2]
                del self.od[-2:]
            self.gp = g
        xi = self.gp if self.skel else 0.5 * (self.gp - self.gr)
        s = S(xi / gref)
        pw = _pow2s(abs(s), beta)
        if self.skel:
            self.sm = abs(s)
        Gt = G0 / (1.0 + (1.0 + beta) * pw)
        ph = pw if self.skel else pm
        hk = hmax * ph / (1.0 + ph)
        tau = G0 * gref * s if self.skel else self.tr + 2.0 * G0 * gref * s
        return tau, Gt, hk


@pytest.mark.parametrize("depth", [1, 3])
def test_stored_skeleton_stress_matches_oracle(depth):
    G0, gref, hmax = 6e7, 1e-3, 0.22
    beta = oracle.ro_beta(hmax)
    rng = np.random.default_rng(41 + depth)
    ev = (C.c_long * 4)()
    worst = np.zeros(3)
    for run in range(6):
        st = oracle.new_spring_mem(depth)
        sp = SmSpring(depth)
        amp = gref * 10.0 ** rng.uniform(-2, 1.5)
        v = 0.0
        for t in range(700):
            v = 0.9 * v + 0.4 * rng.uniform(-1, 1)
            dg = 0.0 if rng.integers(13) == 0 else amp * 0.08 * v
            if rng.integers(61) == 0:
                dg = amp * rng.uniform(-3, 3)  # a jump past the largest strain
            to, Go, ho = oracle.spring_step_mem(st, depth, dg, G0, gref, hmax, ev)
            ts, Gs, hs = sp.step(dg, G0, gref, beta, hmax)
            assert int(st[5]) == sp.skel, (run, t)
            worst = np.maximum(worst, [abs(ts - to) / (G0 * gref), abs(Gs - Go) / G0, abs(hs - ho)])
    assert worst[0] < 1e-12 and worst[1] < 1e-13 and worst[2] < 1e-13, worst
    # the paths take every kind of event: reversals on the skeleton and on
    # branches, rejoins, and with a memory closed inner loops
    assert min(ev[0], ev[1], ev[2]) > 0 and (ev[3] > 0) == (depth > 1), list(ev)
