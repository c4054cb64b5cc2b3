"""Pins of the oracle's extended-precision evaluation (``oracle.fd_exact``: the
same arithmetic in long double, a 64-bit significand) to facts other than
itself: an exact rational solution of the planar double pendulum, and the
double-precision oracle within that one's own error bound."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1609_06779_amd import synth

U64 = 2.0 ** -53


def _double_pendulum(m1, m2, l1, lc1, lc2, i1, i2, g=9.81):
    return synth.Robots(
        n_links=np.array([2], np.int32), axis=np.array([[0, 0, 1.0], [0, 0, 1.0]]),
        home_rot=np.tile(np.eye(3).reshape(9), (2, 1)), offset=np.array([[0, 0, 0.0], [l1, 0, 0]]),
        mass=np.array([m1, m2]), com=np.array([[lc1, 0, 0.0], [lc2, 0, 0]]),
        inertia=np.array([[0.03, 0.04, i1, 0, 0, 0], [0.01, 0.02, i2, 0, 0, 0]]),
        gravity=np.array([0, -g, 0.0]))


@pytest.mark.parametrize("params", [(1.3, 0.7, 0.9, 0.4, 0.35, 0.05, 0.02),
                                    (1.3, 1e-4, 0.9, 0.4, 0.35, 0.05, 1e-7),
                                    (2.0, 0.5, 1.7, 0.85, 1.1, 0.3, 1e-3)])
def test_exact_rational_double_pendulum(params):
    """At q = 0 (sin 0 = 0, cos 0 = 1 exactly) the planar double pendulum's M and
    bias (Euler-Lagrange closed form) are rational in the double parameters, so
    qdd = M^-1 (tau - bias) is a rational number computed exactly here; the
    extended-precision oracle returns it correctly rounded to double (or within
    one unit in the last place)."""
    m1, m2, l1, lc1, lc2, i1, i2 = params
    g = 9.81
    rb = _double_pendulum(m1, m2, l1, lc1, lc2, i1, i2, g)
    rng = np.random.default_rng(11)
    for _ in range(5):
        tau = rng.standard_normal(2)
        qd = rng.uniform(-2, 2, 2)              # velocity terms vanish with sin q2 = 0
        M1, M2, L1, LC1, LC2, I1, I2, G = map(Fraction, (m1, m2, l1, lc1, lc2, i1, i2, g))
        m11 = M1 * LC1 ** 2 + M2 * (L1 ** 2 + LC2 ** 2 + 2 * L1 * LC2) + I1 + I2
        m12 = M2 * (LC2 ** 2 + L1 * LC2) + I2
        m22 = M2 * LC2 ** 2 + I2
        r1 = Fraction(tau[0]) - ((M1 * LC1 + M2 * L1) * G + M2 * LC2 * G)
        r2 = Fraction(tau[1]) - M2 * LC2 * G
        det = m11 * m22 - m12 * m12
        exact = np.array([float((m22 * r1 - m12 * r2) / det), float((-m12 * r1 + m11 * r2) / det)])
        got = oracle.fd_exact(rb, np.zeros(2), qd, tau)
        assert np.all(np.abs(got - exact) <= 2 * U64 * np.abs(exact)), (got, exact)


@pytest.mark.parametrize("n", [4, 16, 64])
def test_exact_agrees_with_double_oracle(n):
    """The double-precision oracle is within its own error bound of the
    extended one, ||qdd - qdd_exact|| <= 16 n cond_2(M) u ||qdd_exact|| (Cholesky's
    backward error times the condition number), and the two agree to a few u
    where M is well conditioned."""
    lengths = [n] * 24
    rb = synth.make_robots(lengths, seed=33, random_home=True)
    q, qd, tau = synth.make_state(lengths, seed=33)
    off = rb.offsets
    d = oracle.fd(rb, q, qd, tau)
    e = oracle.fd_exact(rb, q, qd, tau)
    ms = oracle.crba(rb, q)
    for b, m in enumerate(ms):
        sl = slice(off[b], off[b + 1])
        err = np.linalg.norm(d[sl] - e[sl]) / np.linalg.norm(e[sl])
        assert err <= 16 * n * np.linalg.cond(m) * U64, (n, b, err)
