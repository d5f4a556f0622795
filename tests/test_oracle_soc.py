"""Pins of the oracle's SOC projection (supplementary II-C) against properties the
mathematics fixes: the three cases, idempotence, Moreau decomposition for the
self-dual second-order cone, non-expansiveness, the variational inequality,
positive homogeneity and the 2-D wedge solved geometrically."""
import math

import numpy as np
import pytest

import synth
from oracle import soc


def _rand_cones(seed, n, lo=1, hi=40):
    L = synth.cone_lengths(seed, n, lo, hi)
    off = np.concatenate([[0], np.cumsum(L)])
    x = 3.0 * synth.cone_values(seed + 1, int(off[-1]))
    return x, off


def test_three_cases():
    # inside: unchanged
    t, e = soc.project(2.0, np.array([1.0, 1.0]))
    assert t == 2.0 and np.all(e == [1.0, 1.0])
    # polar cone: origin
    t, e = soc.project(-3.0, np.array([1.0, 2.0]))
    assert t == 0.0 and np.all(e == 0.0)
    # outside: ((t+a)/2, (t+a)/(2a) eta) with a = 5
    t, e = soc.project(1.0, np.array([3.0, 4.0]))
    assert t == pytest.approx(3.0) and np.allclose(e, [1.8, 2.4])
    # boundary a = |t| on both sides and a = 0
    t, e = soc.project(0.0, np.zeros(3))
    assert t == 0.0 and np.all(e == 0.0)
    t, e = soc.project(-1.0, np.zeros(2))
    assert t == 0.0
    # ray (length-1 segment)
    assert soc.project_segments(np.array([-2.0, 3.0]), np.array([0, 1, 2])).tolist() == [0.0, 3.0]


def test_result_in_cone_and_idempotent():
    x, off = _rand_cones(11, 300)
    y = soc.project_segments(x, off)
    for i in range(len(off) - 1):
        a, b = off[i], off[i + 1]
        assert np.linalg.norm(y[a + 1:b]) <= y[a] * (1 + 1e-14) + 1e-300
    z = soc.project_segments(y, off)
    assert np.max(np.abs(z - y)) <= 1e-14 * (1 + np.max(np.abs(y)))


def test_moreau_decomposition():
    # K self-dual: v = Pi_K(v) - Pi_K(-v) and <Pi_K(v), Pi_K(-v)> = 0
    x, off = _rand_cones(12, 300)
    p = soc.project_segments(x, off)
    m = soc.project_segments(-x, off)
    assert np.max(np.abs(x - (p - m))) <= 1e-14 * (1 + np.max(np.abs(x)))
    for i in range(len(off) - 1):
        a, b = off[i], off[i + 1]
        assert abs(p[a:b] @ m[a:b]) <= 1e-13 * (1 + np.linalg.norm(x[a:b]) ** 2)


def test_nonexpansive_and_homogeneous():
    x, off = _rand_cones(13, 200)
    y = x + 0.1 * synth.cone_values(14, x.size)
    px, py = soc.project_segments(x, off), soc.project_segments(y, off)
    for i in range(len(off) - 1):
        a, b = off[i], off[i + 1]
        assert np.linalg.norm(px[a:b] - py[a:b]) <= np.linalg.norm(x[a:b] - y[a:b]) * (1 + 1e-14)
    assert np.allclose(soc.project_segments(2.5 * x, off), 2.5 * px, rtol=1e-14, atol=1e-14)


def test_variational_inequality():
    # <v - Pi v, w - Pi v> <= 0 for w in K
    x, off = _rand_cones(15, 100, 2, 10)
    px = soc.project_segments(x, off)
    w = synth.cone_values(16, x.size)
    for i in range(len(off) - 1):
        a, b = off[i], off[i + 1]
        wi = w[a:b].copy()
        wi[0] = np.linalg.norm(wi[1:]) + abs(wi[0])      # make w a cone member
        assert (x[a:b] - px[a:b]) @ (wi - px[a:b]) <= 1e-12


def test_2d_wedge_geometric():
    # {|y| <= t} is the 90-degree wedge around the t axis; the projection of a point
    # outside both it and its polar lands on the nearest boundary ray.
    for ang in np.linspace(-math.pi, math.pi, 73):
        v = np.array([math.cos(ang), math.sin(ang)]) * 2.0
        t, e = soc.project(v[0], v[1:])
        if abs(v[1]) <= v[0]:
            ref = v
        elif abs(v[1]) <= -v[0]:
            ref = np.zeros(2)
        else:
            ray = np.array([1.0, math.copysign(1.0, v[1])]) / math.sqrt(2.0)
            ref = max(0.0, v @ ray) * ray
        assert np.allclose([t, e[0]], ref, atol=1e-14)


def test_vectorised_rows_match():
    S = 2.0 * synth.cone_values(17, 400 * 9).reshape(400, 9)
    assert np.array_equal(soc.project_rows(S), soc.project_rows_vec(S)) or \
        np.max(np.abs(soc.project_rows(S) - soc.project_rows_vec(S))) <= 1e-15
