"""Pins for the layout metrics of the oracle (no GPU): hand-computed values
on small point sets, the scaling and invariance laws of the definitions, and
the undefined cases."""
import math

import numpy as np

import oracle as O
import synth


def test_node_distribution_unit_square():
    # 4 sides of length 1 and 2 diagonals of squared length 2: 4 + 2/2 = 5
    X = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    assert abs(O.node_distribution(X) - 5.0) < 1e-15
    # scaling by c divides ND by c^2; translation and rotation change nothing
    c, th = 3.0, 0.7
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    Y = (X @ R.T) * c + np.array([5.0, -2.0])
    assert abs(O.node_distribution(Y) - 5.0 / c ** 2) < 1e-12


def test_node_distribution_coincident_pair_is_infinite():
    X = np.array([[0.0, 0.0], [1.0, 2.0], [0.0, 0.0]])
    assert O.node_distribution(X) == math.inf


def test_ulcv_hand_values():
    # a path with edge lengths 1 and 3: mean 2, population std 1 -> 0.5
    X = np.array([[0.0, 0.0], [1.0, 0.0], [4.0, 0.0]])
    assert abs(O.ulcv(X, [0, 1], [1, 2]) - 0.5) < 1e-15
    # lengths 1, 1, 4: mean 2, variance (1 + 1 + 4) / 3 = 2
    X = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [1.0, 5.0]])
    assert abs(O.ulcv(X, [0, 1, 2], [1, 2, 3]) - math.sqrt(2.0) / 2.0) < 1e-15
    # every edge of a regular polygon has the same length
    t = np.linspace(0, 2 * math.pi, 7)[:-1]
    P = np.stack([np.cos(t), np.sin(t)], 1)
    assert O.ulcv(P, np.arange(6), (np.arange(6) + 1) % 6) < 1e-12


def test_ulcv_invariances_and_undefined_cases():
    g = synth.erdos_renyi(60, 5, 3)
    X = synth.uniform_layout(60, 4).astype(np.float64)
    u = O.ulcv(X, g.eu, g.ev)
    assert u > 0
    # scale, translation and edge order do not matter; listing both arcs of
    # every edge does not change mean or deviation
    assert abs(O.ulcv(2.5 * X + 1.0, g.eu, g.ev) - u) < 1e-12
    perm = np.random.default_rng(0).permutation(g.eu.size)
    assert abs(O.ulcv(X, g.ev[perm], g.eu[perm]) - u) < 1e-12
    both_u = np.concatenate([g.eu, g.ev])
    both_v = np.concatenate([g.ev, g.eu])
    assert abs(O.ulcv(X, both_u, both_v) - u) < 1e-12
    assert math.isnan(O.ulcv(X, [], []))
    assert math.isnan(O.ulcv(np.zeros((3, 2)), [0, 1], [1, 2]))
