"""Pins of the two wetting schemes (Sec. II.B, Eqs. 28-33) on single vectors:
closed forms, a brute-force root of the Scheme-I secant line, and the guards."""
import numpy as np
import pytest

import oracle as O


def _unit(v):
    v = np.asarray(v, float)
    return v / np.linalg.norm(v)


def _angle(a, b):
    return np.degrees(np.arccos(np.clip(np.dot(a, b) / np.linalg.norm(a) / np.linalg.norm(b), -1, 1)))


def _rand_pairs(dim, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        nw = _unit(np.r_[rng.standard_normal(dim), np.zeros(3 - dim)])
        nc = _unit(np.r_[rng.standard_normal(dim), np.zeros(3 - dim)])
        if 3.0 < _angle(nc, nw) < 177.0:
            out.append((nc, nw))
    return out


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("theta", [15.0, 30.0, 60.0, 90.0, 120.0, 165.0])
def test_scheme2_hits_theta_exactly_in_plane_of_nc_nw(dim, theta):
    for nc, nw in _rand_pairs(dim, 40, int(theta) + dim):
        out = O.scheme2(dim, nc, nw, theta)
        assert abs(np.linalg.norm(out) - 1) < 1e-14
        assert abs(_angle(out, nw) - theta) < 1e-9
        if dim == 3:
            # coplanar with n_c and n_w
            assert abs(np.dot(out, np.cross(nc, nw))) < 1e-13
        # the kept vector is the one nearer to n_c: on the same side of n_w as n_c
        t = nc - np.dot(nc, nw) * nw
        assert np.dot(out - np.dot(out, nw) * nw, t) > 0


def test_scheme2_keeps_nc_when_parallel_to_wall_normal():
    nw = np.array([0.0, 1.0, 0.0])
    for nc in (nw, -nw):
        assert np.array_equal(O.scheme2(3, nc, nw, 60.0), nc)


def _secant_line_root(nc, nw, theta, s):
    """Brute force: the point v(t) = n_c - t (n_c + s n_w) of the secant line of
    Eqs. (29)-(31) where the angle to n_w is theta, nearest to t = 0 on either
    side (bisection after a fine scan)."""
    c = np.cos(np.radians(theta))
    d = nc + s * nw
    f = lambda t: np.dot(nc - t * d, nw) - np.linalg.norm(nc - t * d) * c
    ts = np.linspace(-0.9, 0.9, 7201)
    fs = np.array([f(t) for t in ts])
    idx = np.where(np.sign(fs[:-1]) != np.sign(fs[1:]))[0]
    if len(idx) == 0:
        return None
    k = idx[np.argmin(np.abs(ts[idx]))]
    a, b = ts[k], ts[k + 1]
    for _ in range(200):
        m = 0.5 * (a + b)
        if np.sign(f(m)) == np.sign(f(a)):
            a = m
        else:
            b = m
    v = nc - 0.5 * (a + b) * d
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("theta", [30.0, 60.0, 90.0, 120.0, 150.0])
def test_scheme1_agrees_with_bisection_root_near_target(dim, theta):
    s = 1 if theta > 90 else -1
    checked = 0
    for nc, nw in _rand_pairs(dim, 60, 11 + dim):
        # near the target angle the three secant steps of Eq. (31) land close to
        # the root of Eq. (28) on the line; a dropped term or a wrong sign in the
        # recurrence would miss it by degrees
        if abs(_angle(nc, nw) - theta) > 8.0:
            continue
        root = _secant_line_root(nc, nw, theta, s)
        assert root is not None
        out = O.scheme1(dim, nc, nw, theta)
        assert np.abs(out - root).max() < 2e-3
        assert abs(_angle(out, nw) - theta) < 0.05
        checked += 1
    assert checked >= 3


def _worst_error(theta, line, dim=2):
    worst = 0.0
    nw = np.array([0.0, 1.0, 0.0])
    for tp in np.arange(5.0, 175.01, 1.0):
        nc = np.array([np.sin(np.radians(tp)), np.cos(np.radians(tp)), 0.0])
        out = O.scheme1(dim, nc, nw, theta, line=line)
        worst = max(worst, abs(_angle(out, nw) - theta))
    return worst


def test_scheme1_line_rule_error_table():
    # With the printed secant start (line = 1) the iteration cannot reach small
    # angles when n_w points into the fluid; the sign rule fixes that.
    assert _worst_error(15.0, 1) > 100.0
    assert _worst_error(15.0, 0) < 11.0
    assert _worst_error(60.0, 0) < 2.0
    assert _worst_error(120.0, 0) < 2.0
    assert _worst_error(90.0, 0) < 1e-6


def test_scheme1_guards():
    nw = np.array([0.0, 1.0, 0.0])
    # parallel / antiparallel to the wall normal: unchanged
    for nc in (nw, -nw):
        assert np.array_equal(O.scheme1(3, nc, nw, 60.0), nc)
    # already at the target angle: f(v0) = 0 -> after the first secant point the
    # iteration stops on |f(v1) - f(v0)| or |f(v1)|, result stays a unit vector
    nc = np.array([np.sin(np.radians(60.0)), np.cos(np.radians(60.0)), 0.0])
    out = O.scheme1(3, nc, nw, 60.0)
    assert abs(np.linalg.norm(out) - 1) < 1e-14
    assert abs(_angle(out, nw) - 60.0) < 1e-6


def test_scheme1_and_2_identical_in_2d_near_target():
    # In 2D both schemes pick the unit vector at angle theta on n_c's side.
    nw = np.array([0.0, 1.0, 0.0])
    for tp in (55.0, 58.0, 63.0, 66.0):
        nc = np.array([np.sin(np.radians(tp)), np.cos(np.radians(tp)), 0.0])
        a = O.scheme1(2, nc, nw, 60.0)
        b = O.scheme2(2, nc, nw, 60.0)
        assert np.abs(a - b).max() < 1e-4
