"""Pins of the oracle's lattice tables, MRT matrix, equilibrium moments,
forcing moments and collision against what the paper prints (Appendix A) and
against identities that hold exactly."""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O


def _read_golden(golden_dir, name):
    rows = []
    with open(os.path.join(golden_dir, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_d3q19_matches_printed_A1_A2(golden_dir):
    rows = _read_golden(golden_dir, "d3q19_lattice_A1_A2.txt")
    tab = {r[0]: r[1:] for r in rows}
    e, w, _ = O.lattice(3)
    for a, key in enumerate(("ex", "ey", "ez")):
        assert [int(x) for x in tab[key]] == list(e[:, a])
    assert np.array_equal(w, np.array([float(Fraction(x)) for x in tab["w"]]))


@pytest.mark.parametrize("dim", [2, 3])
def test_lattice_isotropy(dim):
    e, w, opp = O.lattice(dim)
    q = len(w)
    assert q == (9 if dim == 2 else 19)
    assert abs(w.sum() - 1.0) < 1e-15
    ef = e[:, :dim].astype(float)
    assert np.abs((w[:, None] * ef).sum(0)).max() < 1e-16
    second = np.einsum("i,ia,ib->ab", w, ef, ef)
    assert np.allclose(second, np.eye(dim) / 3.0, atol=1e-16)
    third = np.einsum("i,ia,ib,ic->abc", w, ef, ef, ef)
    assert np.abs(third).max() < 1e-16
    fourth = np.einsum("i,ia,ib,ic,id->abcd", w, ef, ef, ef, ef)
    d = np.eye(dim)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.allclose(fourth, iso, atol=1e-16)
    for i in range(q):
        assert np.array_equal(e[opp[i]], -e[i])


def test_d2q9_is_inplane_subset_of_d3q19():
    e3, _, _ = O.lattice(3)
    e2, w2, _ = O.lattice(2)
    inplane = [i for i in range(19) if e3[i, 2] == 0]
    assert np.array_equal(e2, e3[inplane])
    assert np.allclose(w2, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, rtol=0, atol=1e-17)


def test_mrt_matrix_matches_printed_rows(golden_dir):
    M, _ = O.mrt_matrix()
    rows = _read_golden(golden_dir, "mrt_matrix_A3_printed.txt")
    checked = 0
    for r in rows:
        k = int(r[0])
        if r[1] == "GARBLED":
            continue
        assert [int(x) for x in r[1:]] == list(M[k].astype(int)), k
        checked += 1
    assert checked == 17


def test_mrt_matrix_orthogonal_and_invertible():
    M, n2 = O.mrt_matrix()
    G = M @ M.T
    assert np.array_equal(G, np.diag(np.diag(G)))
    assert np.array_equal(np.diag(G), n2)
    assert list(n2.astype(int)) == [19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8]
    assert np.linalg.matrix_rank(M) == 19
    # The garbled print has rank 18: the rebuilt rows 13/14 are needed.


def _meq_A4(rho, rho0, u):
    """Equilibrium moments as printed in Eq. (A.4), with m_10 = -(3/2) p_xx^eq read
    from its label (the printed right-hand side multiplies 3 p_xx^eq instead)."""
    ux, uy, uz = u
    usq = ux * ux + uy * uy + uz * uz
    pxx3 = rho0 * (2 * ux * ux - uy * uy - uz * uz)
    pww = rho0 * (uy * uy - uz * uz)
    return np.array([
        rho, -11 * rho + 19 * rho0 * usq, 3 * rho - 5.5 * rho0 * usq,
        rho0 * ux, -2 / 3 * rho0 * ux, rho0 * uy, -2 / 3 * rho0 * uy, rho0 * uz, -2 / 3 * rho0 * uz,
        pxx3, -0.5 * pxx3, pww, -0.5 * pww,
        rho0 * ux * uy, rho0 * uy * uz, rho0 * ux * uz, 0.0, 0.0, 0.0])


@pytest.mark.parametrize("seed", range(5))
def test_meq_equals_printed_A4(seed):
    rng = np.random.default_rng(seed)
    rho = 1 + 0.1 * rng.standard_normal()
    u = 0.05 * rng.standard_normal(3)
    got = O.meq(rho, 1.0, u)
    assert np.allclose(got, _meq_A4(rho, 1.0, u), rtol=0, atol=1e-14)


def _sf_A5(u, F, S):
    """Forcing moments as printed in Eq. (A.5)."""
    ux, uy, uz = u
    Fx, Fy, Fz = F
    uF = ux * Fx + uy * Fy + uz * Fz
    h = lambda k: 1 - 0.5 * S[k]
    return np.array([
        0, 38 * h(1) * uF, -11 * h(2) * uF, Fx, -2 / 3 * h(4) * Fx, Fy, -2 / 3 * h(6) * Fy, Fz, -2 / 3 * h(8) * Fz,
        2 * h(9) * (2 * ux * Fx - uy * Fy - uz * Fz), h(10) * (-2 * ux * Fx + uy * Fy + uz * Fz),
        2 * h(11) * (uy * Fy - uz * Fz), h(12) * (-uy * Fy + uz * Fz),
        h(13) * (uy * Fx + ux * Fy), h(14) * (uz * Fy + uy * Fz), h(15) * (ux * Fz + uz * Fx), 0, 0, 0])


@pytest.mark.parametrize("seed", range(5))
def test_forcing_moments_equal_printed_A5(seed):
    rng = np.random.default_rng(100 + seed)
    u = 0.05 * rng.standard_normal(3)
    F = 1e-3 * rng.standard_normal(3)
    s_nu, s_q = O.rates(rng.uniform(-1, 1), 1.0, 0.6)
    S = np.array([0, s_nu, s_nu, 0, s_q, 0, s_q, 0, s_q, s_nu, s_nu, s_nu, s_nu, s_nu, s_nu, s_nu, s_q, s_q, s_q])
    assert np.allclose(O.forcing_moments(u, F, S), _sf_A5(u, F, S), rtol=0, atol=1e-15)


@pytest.mark.parametrize("phi", [-1.0, -0.3, 0.0, 0.7, 1.0])
@pytest.mark.parametrize("taus", [(1.0, 0.6), (0.6, 1.0), (1.0, 1.0), (0.9, 1.7)])
def test_rates_eq13_to_16(phi, taus):
    tr, tb = taus
    s_nu, s_q = O.rates(phi, tr, tb)
    nu_r, nu_b = (tr - 0.5) / 3, (tb - 0.5) / 3
    # harmonic mean, Eq. (14): pure phases recover their own viscosity
    if phi == 1.0:
        assert abs(1 / s_nu - 0.5 - 3 * nu_r) < 1e-14
    if phi == -1.0:
        assert abs(1 / s_nu - 0.5 - 3 * nu_b) < 1e-14
    # Eq. (16) makes the "magic" product (1/S_nu - 1/2)(1/S_q - 1/2) equal 3/16
    assert abs((1 / s_nu - 0.5) * (1 / s_q - 0.5) - 3 / 16) < 1e-14


def _rand_node(rng, q=19):
    e, w, _ = O.lattice(3 if q == 19 else 2)
    f = w * (1 + 0.05 * rng.standard_normal(q))
    return f


@pytest.mark.parametrize("seed", range(4))
def test_mrt_with_equal_rates_is_bgk(seed):
    rng = np.random.default_rng(seed)
    f = _rand_node(rng)
    rho = f.sum()
    u = 0.03 * rng.standard_normal(3)
    F = 1e-3 * rng.standard_normal(3)
    s = 1 / 0.8
    bgk = O.collide_node(3, 0, f, rho, 1.0, u, F, s, s)
    mrt = O.collide_node(3, 1, f, rho, 1.0, u, F, s, s, S=np.full(19, s))
    assert np.abs(bgk - mrt).max() < 1e-15


@pytest.mark.parametrize("collision", [0, 1])
def test_collision_conserves_mass_and_adds_force(collision):
    rng = np.random.default_rng(7)
    e, w, _ = O.lattice(3)
    f = _rand_node(rng)
    rho = f.sum()
    F = 1e-3 * rng.standard_normal(3)
    j = e.T.astype(float) @ f
    u = (j + 0.5 * F) / rho
    s_nu, s_q = O.rates(0.2, 1.0, 0.6)
    out = O.collide_node(3, collision, f, rho, 1.0, u, F, s_nu, s_q)
    assert abs(out.sum() - rho) < 1e-15
    if collision == 1:
        # conserved moments have zero rate: momentum changes by exactly F
        assert np.allclose(e.T.astype(float) @ out, j + F, rtol=0, atol=1e-16)


@pytest.mark.parametrize("dim,collision", [(2, 0), (3, 0), (3, 1)])
def test_rest_state_is_a_fixed_point(dim, collision):
    e, w, _ = O.lattice(dim)
    for rho in (1.0, 0.97):
        f = w * rho
        s_nu, s_q = O.rates(0.0, 1.0, 0.6)
        out = O.collide_node(dim, collision, f, rho, 1.0, np.zeros(3), np.zeros(3), s_nu, s_q)
        assert np.abs(out - f).max() < 1e-16
