"""Pins of the oracle's zero-momentum single-baryon two-point functions
(Eq. (1) with one baryon at sink and source, operators of Eqs. (2)-(3),
blocks of Eq. (5)):

- the textbook Wick contractions of eps (q Cg5 q') q'' written directly on
  the propagators (no normal blocks, no permutation enumeration): the proton
  form (identical quarks 1 and 3) and the cascade form (identical quarks 2
  and 3), which the oracle must reproduce for p, n, Sigma+, Xi0;
- the SU(3) limit S_u = S_d = S_s, where the eight octet operators are one
  multiplet and every diagonal two-point function is the same;
- the isospin limit S_u = S_d, where Lambda (I = 0) and Sigma0 (I = 1) do
  not mix, while they do with independent u and d."""
import numpy as np
import pytest

import oracle

L = (2, 2, 2)
OCTET = ["p", "n", "Lambda", "Sigma+", "Sigma0", "Sigma-", "Xi0", "Xi-"]


def props(seed):
    rng = np.random.default_rng(seed)
    V = int(np.prod(L))
    return [(rng.standard_normal((V, 12, 12)) + 1j * rng.standard_normal((V, 12, 12))) / np.sqrt(2)
            for _ in range(3)]


def eps3():
    e = np.zeros((3, 3, 3))
    for a, b, c, s in ((0, 1, 2, 1), (1, 2, 0, 1), (2, 0, 1, 1), (0, 2, 1, -1), (2, 1, 0, -1), (1, 0, 2, -1)):
        e[a, b, c] = s
    return e


def spin_colour(S):
    """[x, sink spin, sink colour, source spin, source colour]"""
    return S.reshape(-1, 4, 3, 4, 3)


def textbook(SA, SB, identical):
    """eps_abc (A_a Cg5 B_b) X_c at sink and source, X = A (identical = 13)
    or X = B (identical = 23): the direct term minus the exchange of the two
    identical quarks; sink quarks (u, a), (v, b), (l, c), source quarks
    (s, d), (t, e), (m, f) with Cg5 on the first two spins of each side and
    the third spins l, m the open indices."""
    A, B = spin_colour(SA), spin_colour(SB)
    e, g = eps3(), oracle.cg5()
    X = A if identical == 13 else B
    direct = np.einsum('abc,uv,def,st,xuasd,xvbte,xlcmf->lm', e, g, e, g, A, B, X, optimize=True)
    if identical == 13:
        exch = np.einsum('abc,uv,def,st,xuamf,xvbte,xlcsd->lm', e, g, e, g, A, B, A, optimize=True)
    else:
        exch = np.einsum('abc,uv,def,st,xuasd,xvbmf,xlcte->lm', e, g, e, g, A, B, B, optimize=True)
    return (direct - exch)[:2, :2]


def test_two_point_matches_textbook_contractions():
    Su, Sd, Ss = S = props(11)
    C = oracle.two_point(L, S, [("p", "p"), ("n", "n"), ("Sigma+", "Sigma+"), ("Xi0", "Xi0"), ("Xi-", "Xi-")])
    want = [textbook(Su, Sd, 13),   # p = eps (u Cg5 d) u
            textbook(Su, Sd, 23),   # n = -eps (u Cg5 d) d, weight squared
            textbook(Su, Ss, 13),   # Sigma+ = -eps (u Cg5 s) u
            textbook(Su, Ss, 23),   # Xi0 = eps (u Cg5 s) s
            textbook(Sd, Ss, 23)]   # Xi- = -eps (d Cg5 s) s
    for k, w in enumerate(want):
        assert np.abs(w).max() > 1.0
        np.testing.assert_allclose(C[k], w, rtol=0, atol=1e-11 * np.abs(w).max())


def test_su3_limit_octet_is_one_multiplet():
    Su = props(12)[0]
    C = oracle.two_point(L, [Su, Su, Su], [(b, b) for b in OCTET])
    assert np.abs(C[0]).max() > 1.0
    for k in range(1, 8):
        np.testing.assert_allclose(C[k], C[0], rtol=0, atol=1e-12 * np.abs(C[0]).max(), err_msg=OCTET[k])


def test_isospin_limit_lambda_sigma0_do_not_mix():
    Su, Sd, Ss = props(13)
    mix = [("Lambda", "Sigma0"), ("Sigma0", "Lambda")]
    iso = oracle.two_point(L, [Su, Su, Ss], mix + [("Lambda", "Lambda")])
    scale = np.abs(iso[2]).max()
    assert scale > 1.0
    assert np.abs(iso[:2]).max() < 1e-12 * scale
    gen = oracle.two_point(L, [Su, Sd, Ss], mix)
    assert np.abs(gen).max() > 1e-3 * scale


def test_two_point_rejects_unknown_operator():
    with pytest.raises(RuntimeError):
        oracle.two_point(L, props(14), [(11, 0)])
