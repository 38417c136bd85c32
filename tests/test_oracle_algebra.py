"""Pins of the oracle's lattice algebra against what the paper prints and what
mathematics fixes (no GPU).

* The printed matrices of App. A (P, P^-1) and App. B (F, F^-1) are read from
  ``tests/golden/paper_matrices.json`` (transcribed as printed) and compared
  with the oracle, which never uses them: it takes central moments by the
  definition sum of Eq. cmscalar and inverts them with a linear solve.
* Rest weights, the shift identity F(u)^-1 = F(-u), the collision's conserved
  moments and the momentum source of App. D are checked as identities.
"""
import json
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_matrices.json")


def _load():
    with open(GOLD) as fh:
        return json.load(fh)


def _eval_matrix(rows, ux, uy):
    from fractions import Fraction  # noqa: F401  (entries such as "1/2")
    env = {"ux": ux, "uy": uy, "__builtins__": {}}
    return np.array([[float(eval(str(e), env)) for e in r] for r in rows])


def _def_matrix(oracle, ux, uy):
    """M(u)[k, a] = central moment k of a unit population in direction a."""
    eye = np.eye(9)
    return np.array([oracle.central_moments(eye[a], ux, uy) for a in range(9)]).T


def test_directions_and_printed_ex_typo(oracle_mod):
    g = _load()
    ex, ey = oracle_mod.directions()
    assert list(ey) == g["ey"]
    # printed ex differs only in the last entry; row 1 of the printed P fixes it
    diff = [i for i in range(9) if ex[i] != g["ex"][i]]
    assert diff == [8]
    assert list(ex) == g["P"][1]


def test_P_matches_definition_and_printed_inverse(oracle_mod):
    g = _load()
    P = np.array(g["P"], dtype=float)
    M0 = _def_matrix(oracle_mod, 0.0, 0.0)
    assert np.array_equal(M0, P)
    Pinv = _eval_matrix(g["Pinv"], 0.0, 0.0)
    assert np.array_equal(P @ Pinv, np.eye(9))
    assert np.array_equal(Pinv @ P, np.eye(9))


def test_rest_weights(oracle_mod):
    w = oracle_mod.weights()
    expect = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    assert np.allclose(w, expect, rtol=0, atol=5e-16)
    assert abs(w.sum() - 1.0) < 1e-15


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_F_against_definition(oracle_mod, seed):
    """F(u) = M(u) P^-1.  All printed entries agree except row 8, columns 1
    and 2, where the definition gives twice the printed value."""
    g = _load()
    rng = np.random.default_rng(seed)
    ux, uy = rng.uniform(-0.3, 0.3, 2)
    P = np.array(g["P"], dtype=float)
    F_def = _def_matrix(oracle_mod, ux, uy) @ np.linalg.inv(P)
    F_pr = _eval_matrix(g["F"], ux, uy)
    bad = np.argwhere(~np.isclose(F_def, F_pr, rtol=1e-13, atol=1e-15))
    assert sorted(map(tuple, bad)) == [(8, 1), (8, 2)]
    assert np.isclose(F_def[8, 1], 2 * F_pr[8, 1], rtol=1e-13)
    assert np.isclose(F_def[8, 2], 2 * F_pr[8, 2], rtol=1e-13)
    Finv_pr = _eval_matrix(g["Finv"], ux, uy)
    Finv_def = np.linalg.inv(F_def)
    bad = np.argwhere(~np.isclose(Finv_def, Finv_pr, rtol=1e-12, atol=1e-15))
    assert sorted(map(tuple, bad)) == [(8, 1), (8, 2)]
    # corrected printed pair is an exact inverse pair; printed pair is not
    Fc, Fic = F_pr.copy(), Finv_pr.copy()
    Fc[8, 1:3] *= 2
    Fic[8, 1:3] *= 2
    assert np.allclose(Fc @ Fic, np.eye(9), atol=1e-15)
    err = F_pr @ Finv_pr - np.eye(9)
    assert abs(err[8, 0] - 2 * ux * ux * uy * uy) < 1e-15


@pytest.mark.parametrize("seed", [3, 4])
def test_shift_identity(oracle_mod, seed):
    """Central moments about u of populations rebuilt from central moments
    about u are the input (solve round trip), and F(u)^-1 = F(-u)."""
    rng = np.random.default_rng(seed)
    ux, uy = rng.uniform(-0.2, 0.2, 2)
    k = rng.standard_normal(9)
    q = oracle_mod.populations_from_central(k, ux, uy)
    assert np.allclose(oracle_mod.central_moments(q, ux, uy), k, atol=1e-14)
    P = _def_matrix(oracle_mod, 0, 0)
    F = _def_matrix(oracle_mod, ux, uy) @ np.linalg.inv(P)
    Fm = _def_matrix(oracle_mod, -ux, -uy) @ np.linalg.inv(P)
    assert np.allclose(F @ Fm, np.eye(9), atol=1e-15)


@pytest.mark.parametrize("seed", [5, 6, 7])
def test_scalar_collision_against_printed_matrices(oracle_mod, seed):
    """Collision of App. C / Sec. 3 evaluated with the printed P, the printed
    P^-1 and the row-8-corrected F, F^-1 matches the oracle (definition sum +
    solve)."""
    g = _load()
    rng = np.random.default_rng(seed)
    ux, uy = rng.uniform(-0.1, 0.1, 2)
    q = rng.uniform(0.0, 0.2, 9)
    s = q.sum()
    jx, jy = rng.uniform(-0.01, 0.01, 2)
    w1 = 1.7
    P = np.array(g["P"], dtype=float)
    Pinv = _eval_matrix(g["Pinv"], 0, 0)
    F = _eval_matrix(g["F"], ux, uy)
    Finv = _eval_matrix(g["Finv"], ux, uy)
    F[8, 1:3] *= 2
    Finv[8, 1:3] *= 2
    k = F @ (P @ q)
    keq = np.array([s, jx, jy, s / 3, s / 3, 0, 0, 0, s / 9])
    lam = np.array([1, w1, w1, 1, 1, 1, 1, 1, 1.0])
    kt = k + lam * (keq - k)
    ref = Pinv @ (Finv @ kt)
    out = oracle_mod.collide_scalar(q, ux, uy, s, jx, jy, w1)
    assert np.allclose(out, ref, rtol=1e-13, atol=1e-15)
    # zeroth moment conserved; first moment relaxes as stated
    assert abs(out.sum() - s) < 1e-15
    ex, ey = oracle_mod.directions()
    k10 = np.dot(q, ex - ux)
    k10_post = np.dot(out, ex - ux)
    assert abs(k10_post - ((1 - w1) * k10 + w1 * jx)) < 1e-14


@pytest.mark.parametrize("seed", [8, 9])
def test_flow_collision_moments(oracle_mod, seed):
    """App. D: with u defined by cs2 rho u = sum e g + cs2 F_t/2 the collision
    adds exactly cs2 F_t to the first raw moment and sigma_00 to the zeroth;
    with the equilibria's first-order entries -psi u the post-collision raw
    first moment is rho cs2 u + cs2 F_t/2."""
    rng = np.random.default_rng(seed)
    cs2 = 1 / 3
    rho = rng.uniform(0.8, 1.2)
    w = oracle_mod.weights()
    ex, ey = oracle_mod.directions()
    g = w * (rho * cs2 + 1e-3 * rng.standard_normal(9))
    ftx, fty = 1e-4 * rng.standard_normal(2)
    fpx, fpy = 1e-4 * rng.standard_normal(2)
    jx, jy = np.dot(g, ex), np.dot(g, ey)
    ux = (jx + 0.5 * cs2 * ftx) / (cs2 * rho)
    uy = (jy + 0.5 * cs2 * fty) / (cs2 * rho)
    gam = fpx * ux + fpy * uy
    P = g.sum() + 0.5 * gam
    out = oracle_mod.collide_flow(g, ux, uy, P, rho, fpx, fpy, ftx, fty, 1.0, 1.3)
    assert abs(np.dot(out, ex) - jx - cs2 * ftx) < 1e-15
    assert abs(np.dot(out, ey) - jy - cs2 * fty) < 1e-15
    assert abs(out.sum() - g.sum() - gam) < 1e-15
    assert abs(np.dot(out, ex) - (rho * cs2 * ux + 0.5 * cs2 * ftx)) < 1e-15


def test_flow_equilibrium_raw_moments(oracle_mod):
    """With no force and g at its equilibrium, the raw moments are
    (P, rho cs2 u, cs2 (P + rho ux^2), ...): the reading -psi u of the
    first-order entries.  The printed +psi u would give (2P - rho cs2) u."""
    cs2 = 1 / 3
    rho, P, ux, uy = 1.1, 0.4, 0.03, -0.02
    psi = P - rho * cs2
    eq = [P, -psi * ux, -psi * uy, cs2 * P + psi * ux ** 2, cs2 * P + psi * uy ** 2,
          psi * ux * uy, -psi * (ux ** 2 + cs2) * uy, -psi * (uy ** 2 + cs2) * ux,
          cs2 ** 3 * rho + psi * (ux ** 2 + cs2) * (uy ** 2 + cs2)]
    g = oracle_mod.populations_from_central(eq, ux, uy)
    ex, ey = oracle_mod.directions()
    assert abs(np.dot(g, ex) - rho * cs2 * ux) < 1e-15
    assert abs(np.dot(g, ey) - rho * cs2 * uy) < 1e-15
    assert abs(np.dot(g, ex * ex) - cs2 * (P + rho * ux * ux)) < 1e-15
    assert abs(np.dot(g, ex * ey) - cs2 * rho * ux * uy) < 1e-15
    # a fixed point of the unforced collision
    out = oracle_mod.collide_flow(g, ux, uy, P, rho, 0, 0, 0, 0, 1.0, 1.4)
    assert np.allclose(out, g, atol=1e-15)


def test_langmuir_special_cases(oracle_mod):
    """Eq. EOS: sigma(0) = sigma0; beta = 0 is clean; sigma vanishes at
    c/c_max = 1 - exp(-1/beta); strictly decreasing in c."""
    s0, b, cm = 0.01, 0.25, 1.0
    assert oracle_mod.langmuir(s0, b, cm, 0.0) == s0
    assert oracle_mod.langmuir(s0, 0.0, cm, 0.7) == s0
    c0 = cm * (1 - np.exp(-1 / b))
    assert abs(oracle_mod.langmuir(s0, b, cm, c0)) < 1e-17
    vals = [oracle_mod.langmuir(s0, b, cm, c) for c in np.linspace(0, 0.9, 10)]
    assert all(x > y for x, y in zip(vals, vals[1:]))
    # small-c slope: d sigma/dc = -sigma0 beta / c_max
    eps = 1e-7
    slope = (oracle_mod.langmuir(s0, b, cm, eps) - s0) / eps
    assert abs(slope + s0 * b / cm) < 1e-8


def test_transport_relations(oracle_mod):
    """D = cs2 (1/omega - 1/2) (Eq. diffcoeffscalarfield and App. C/D)."""
    for d in (0.01, 0.1, 1 / 6, 0.5):
        w = oracle_mod.omega_from_transport(d)
        assert abs((1 / 3) * (1 / w - 0.5) - d) < 1e-15
