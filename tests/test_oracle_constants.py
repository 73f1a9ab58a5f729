"""Pins of the oracle's lattice constants and per-node formulas.

Each test checks the oracle against something the paper or the mathematics
fixes independently of the oracle's own code: isotropy conditions solved in
exact rational arithmetic, the exact moments the equilibrium and the Guo
forcing term are built to have, the two printed forms of the local adhesion
parameter (Eq. 11 and Eq. 12), and the printed Table 1.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _solve_rational(A, b):
    """Gauss-Jordan elimination over the rationals; returns the unique
    solution or raises if the system is singular."""
    n = len(A)
    M = [list(map(Fraction, row)) + [Fraction(bv)] for row, bv in zip(A, b)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                fct = M[r][col] / M[col][col]
                M[r] = [a - fct * c for a, c in zip(M[r], M[col])]
    return [M[r][n] / M[r][r] for r in range(n)]


def test_e8_weights_follow_from_isotropy(oracle_mod):
    """P1 -- Sec. 2.4 uses eighth-order isotropy.  The five shell weights
    W(1), W(2), W(4), W(5), W(8) of the 24-position stencil are fixed by:
    sum W e_x^2 = 1 and isotropy of the 4th, 6th and 8th moment tensors
    (2-D isotropic tensors: T_xxxx = 3 T_xxyy, T_x6 = 5 T_x4y2,
    T_x8 = 7 T_x6y2, 3 T_x6y2 = 5 T_x4y4).  Solved here in rationals."""
    shells = {1: [(1, 0), (0, 1), (-1, 0), (0, -1)],
              2: [(1, 1), (-1, 1), (-1, -1), (1, -1)],
              4: [(2, 0), (0, 2), (-2, 0), (0, -2)],
              5: [(2, 1), (1, 2), (-1, 2), (-2, 1), (-2, -1), (-1, -2), (1, -2), (2, -1)],
              8: [(2, 2), (-2, 2), (-2, -2), (2, -2)]}
    keys = [1, 2, 4, 5, 8]

    def mom(p, q):
        return [sum(Fraction(ex) ** p * Fraction(ey) ** q for ex, ey in shells[s]) for s in keys]

    rows = [mom(2, 0),
            [a - 3 * b for a, b in zip(mom(4, 0), mom(2, 2))],
            [a - 5 * b for a, b in zip(mom(6, 0), mom(4, 2))],
            [a - 7 * b for a, b in zip(mom(8, 0), mom(6, 2))],
            [3 * a - 5 * b for a, b in zip(mom(6, 2), mom(4, 4))]]
    sol = dict(zip(keys, _solve_rational(rows, [1, 0, 0, 0, 0])))
    assert sol == {1: Fraction(4, 21), 2: Fraction(4, 45), 4: Fraction(1, 60),
                   5: Fraction(2, 315), 8: Fraction(1, 5040)}

    ex, ey, W, _ = oracle_mod.e8()
    pos = set(zip(ex.tolist(), ey.tolist()))
    assert len(pos) == 24
    assert pos == {p for s in keys for p in shells[s]}
    for x, y, w in zip(ex, ey, W):
        assert w == float(sol[int(x * x + y * y)])
    # odd moments vanish, even moments isotropic (numerically, as a cross-check)
    for p, q in [(1, 0), (0, 1), (3, 0), (2, 1), (1, 2), (5, 0), (3, 3)]:
        assert abs(np.sum(W * ex ** p * ey ** q)) < 1e-15
    assert abs(np.sum(W * ex ** 2) - 1.0) < 1e-15


def test_table1_copy_map(oracle_mod):
    """Table 1 (Sec. 2.4): second-layer node n is copied from n-8, n-12 or
    n-16.  With the numbering used here this sends every second-layer
    position to the first-layer position in the same direction
    (sign(e_x), sign(e_y)), and the printed example 24 <- 8 holds."""
    ex, ey, W, cp = oracle_mod.e8()
    for lo, hi, off in GOLDEN["table1_second_to_first"]["value"]:
        for n in range(lo, hi + 1):
            assert cp[n - 1] == n + off - 1
    assert all(cp[:8] == -1)
    for n in range(8, 24):
        m = cp[n]
        assert (ex[m], ey[m]) == (np.sign(ex[n]), np.sign(ey[n]))
    a, b = GOLDEN["table1_worked_example"]["value"]
    assert cp[a - 1] == b - 1
    # the first layer is the D2Q9 link set in the same order
    qx, qy, _, _ = oracle_mod.d2q9()
    assert list(zip(ex[:8], ey[:8])) == list(zip(qx[1:], qy[1:]))


def test_d2q9_moments(oracle_mod):
    """P2 -- D2Q9 weights: sum w = 1, sum w e e = I/3,
    sum w e_a e_b e_c e_d = (d_ab d_cd + d_ac d_bd + d_ad d_bc) / 9, odd moments 0."""
    ex, ey, w, opp = oracle_mod.d2q9()
    E = np.stack([ex, ey], 1).astype(float)
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose(np.einsum("i,ia,ib->ab", w, E, E), np.eye(2) / 3, atol=1e-15)
    d = np.eye(2)
    iso4 = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
            + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, E, E, E, E), iso4, atol=1e-15)
    assert np.allclose(np.einsum("i,ia->a", w, E), 0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, E, E, E), 0, atol=1e-16)
    for i in range(9):
        assert (ex[opp[i]], ey[opp[i]]) == (-ex[i], -ey[i])


def test_equilibrium_moments(oracle_mod):
    """Eq. 6 is built so that sum f^eq = rho, sum f^eq e = rho u and
    sum f^eq e e = rho (u u + I/3) hold exactly on D2Q9."""
    ex, ey, _, _ = oracle_mod.d2q9()
    E = np.stack([ex, ey], 1).astype(float)
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = rng.uniform(0.01, 2.0)
        u = rng.uniform(-0.2, 0.2, 2)
        feq = oracle_mod.equilibrium(rho, u)
        assert abs(feq.sum() - rho) < 1e-14
        assert np.allclose(E.T @ feq, rho * u, atol=1e-15)
        assert np.allclose(np.einsum("i,ia,ib->ab", feq, E, E),
                           rho * (np.outer(u, u) + np.eye(2) / 3), atol=1e-14)


def test_guo_forcing_moments(oracle_mod):
    """P3 -- Eq. 7 (Guo's term) has zeroth moment 0, first moment F and
    second moment u F + F u."""
    ex, ey, _, _ = oracle_mod.d2q9()
    E = np.stack([ex, ey], 1).astype(float)
    rng = np.random.default_rng(2)
    for _ in range(20):
        F = rng.uniform(-1e-2, 1e-2, 2)
        u = rng.uniform(-0.2, 0.2, 2)
        Fi = oracle_mod.forcing(F, u)
        assert abs(Fi.sum()) < 1e-17
        assert np.allclose(E.T @ Fi, F, rtol=0, atol=1e-17)
        assert np.allclose(np.einsum("i,ia,ib->ab", Fi, E, E),
                           np.outer(u, F) + np.outer(F, u), rtol=0, atol=1e-17)


@pytest.mark.parametrize("Gw1,Gw2", [(1.3, 0.9), (0.234, 0.9), (0.9, 0.9), (2.0, 0.5)])
def test_local_adhesion_eq11(oracle_mod, Gw1, Gw2):
    """P4 -- Eq. 11: G(x) = G_w1 above delta, G_w2 below -delta, the
    harmonic mean at rho^e = 0, and the quadratic pieces meet the constant
    pieces with zero slope (C1 continuity)."""
    delta = GOLDEN["delta"]["value"]
    G = lambda r: oracle_mod.local_G(r, Gw1, Gw2, delta)
    hm = 2 * Gw1 * Gw2 / (Gw1 + Gw2)
    assert G(0.95) == Gw1 and G(-0.95) == Gw2
    assert abs(G(delta) - Gw1) < 1e-14
    assert abs(G(-delta) - Gw2) < 1e-14
    assert abs(G(0.0) - hm) < 1e-15
    assert abs(G(1e-12) - hm) < 1e-10
    for h in (1e-3, 1e-4):
        # value gap O(h^2) from both sides => zero slope at the joins
        assert abs(G(delta - h) - Gw1) < 4 * abs(Gw1 - hm) / delta ** 2 * h * h + 1e-14
        assert abs(G(-delta + h) - Gw2) < 4 * abs(Gw2 - hm) / delta ** 2 * h * h + 1e-14
        # continuity at 0 with matching slopes from each side: the one-sided
        # slopes are s2 and t2, both equal to 2 (G_w1 - hm) / delta ... only
        # when G_w1 - hm = hm - G_w2; in general just continuity.
        assert abs(G(h) - G(-h)) < 10 * h * (abs(Gw1) + abs(Gw2))
    # monotone between the two plateaus
    r = np.linspace(-1, 1, 401)
    g = np.array([G(v) for v in r])
    dg = np.diff(g)
    assert np.all(dg * np.sign(Gw1 - Gw2) >= -1e-15)


@pytest.mark.parametrize("lam", [0.26, 0.35, 0.47, 0.88, 1.0, 1.35, 2.1])
def test_local_adhesion_eq12_lambda_form(oracle_mod, lam):
    """P4 -- Eq. 12 with its primed coefficients (printed in Sec. 2.3.2)
    equals Eq. 11 divided by G_w2, with lambda = G_w1 / G_w2."""
    delta = GOLDEN["delta"]["value"]
    Gw2 = 0.9
    Gw1 = lam * Gw2
    s1 = t1 = 2 * lam / (1 + lam)
    s2 = 2 * (lam ** 2 - lam) / (delta * (1 + lam))
    s3 = (lam - lam ** 2) / (delta ** 2 * (1 + lam))
    t2 = 2 * (lam - 1) / (delta * (1 + lam))
    t3 = (lam - 1) / (delta ** 2 * (1 + lam))
    for r in np.linspace(-1, 1, 81):
        if r > delta:
            ref = lam
        elif r > 0:
            ref = s1 + s2 * r + s3 * r * r
        elif r > -delta:
            ref = t1 + t2 * r + t3 * r * r
        else:
            ref = 1.0
        assert abs(oracle_mod.local_G(r, Gw1, Gw2, delta) / Gw2 - ref) < 1e-13
    if lam == 1.0:
        for r in np.linspace(-1, 1, 21):
            assert abs(oracle_mod.local_G(r, Gw1, Gw2, delta) - Gw2) < 1e-15


def test_fig6_parameters_support_Gw2_equals_G12():
    """Reading of the adhesion mapping: the original-scheme G_w1 values of
    Fig. 6 (a-e) are lambda * G12 for the improved-scheme lambdas of
    Fig. 6 (f-j), i.e. G_w2 = G12 in both schemes (Sec. 2.3.2 states
    G_w2 = G12)."""
    g = GOLDEN
    for gw1, lam in zip(g["original_Gw1"]["value"], g["improved_lambda"]["value"]):
        assert abs(gw1 - lam * g["G12_cylinder"]["value"]) < 0.0021
