"""Pins for the exact channel-representation arithmetic (Sec. 4.1): R(P), the trace
formula, the sparse column rule, products, orthogonality, Cliffords and bounds."""

import numpy as np
import pytest

import seeded_inputs
from oracle import cyclotomic as cy
from oracle import pauli, zmat


def zmat_from_trace(u, n):
    A, B, e = cy.channel_rep_trace(u, n)
    return zmat.ZMat(A, B, e).reduce()


def test_R_of_Z_is_T_gate():
    # n = 1: R(Z) = diag(1, omega) exactly
    t = cy.rotation(2, 1)
    expect = cy.CycMat([[[1, 0], [0, 0]], [[0, 0], [0, 1]], [[0, 0], [0, 0]], [[0, 0], [0, 0]]], 0)
    assert t.equals(expect)


@pytest.mark.parametrize("n", [1, 2])
def test_R_pow8_is_identity(n):
    ident = cy.CycMat.identity(n)
    for p in range(1, 4 ** n):
        r = cy.rotation(p, n)
        acc = ident
        for _ in range(8):
            acc = acc @ r
        assert acc.equals(ident), p


@pytest.mark.parametrize("n", [1, 2])
def test_R_matches_exponential_closed_form(n):
    # R(P) = e^{i pi/8} exp(-i pi/8 P) = e^{i pi/8} (cos(pi/8) I - i sin(pi/8) P)
    th = np.pi / 8
    for p in range(1, 4 ** n):
        pm = pauli.matrix(p, n)
        expect = np.exp(1j * th) * (np.cos(th) * np.eye(2 ** n) - 1j * np.sin(th) * pm)
        assert np.allclose(cy.rotation(p, n).to_complex(), expect, atol=1e-12)


@pytest.mark.parametrize("n", [1, 2])
def test_column_rule_matches_trace_formula(n):
    for p in range(1, 4 ** n):
        via_trace = zmat_from_trace(cy.rotation(p, n), n)
        assert via_trace.equals(zmat.rot_hat(p, n)), p


def test_column_rule_matches_trace_formula_n3_spot():
    n = 3
    for p in (5, 42):
        assert zmat_from_trace(cy.rotation(p, n), n).equals(zmat.rot_hat(p, n))


@pytest.mark.parametrize("n", [1, 2])
def test_homomorphism_of_channel_rep(n):
    # (U V)^ = U^ V^ on seeded products of rotations
    rng = np.random.default_rng(10 + n)
    for _ in range(4):
        ps = [int(v) for v in rng.integers(1, 4 ** n, 3)]
        u = cy.CycMat.identity(n)
        for p in ps:
            u = u @ cy.rotation(p, n)
        lhs = zmat_from_trace(u, n)
        rhs = zmat.ZMat.identity(n)
        for p in ps:
            rhs = rhs @ zmat.rot_hat(p, n)
        assert lhs.equals(rhs)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_right_rot_equals_dense_product(n):
    rng = np.random.default_rng(20 + n)
    m = zmat.product_of_rotations([int(v) for v in rng.integers(1, 4 ** n, 4)], n)
    for p in [int(v) for v in rng.integers(1, 4 ** n, 3)]:
        assert m.right_rot(p, n).equals(m @ zmat.rot_hat(p, n))
        assert m.right_rot(p, n, transpose=True).equals(m @ zmat.rot_hat(p, n).T())


@pytest.mark.parametrize("n", [1, 2, 3])
def test_rotation_powers(n):
    for p in range(1, 4 ** n, max(1, (4 ** n) // 9)):
        r = zmat.rot_hat(p, n)
        r2 = r @ r
        assert r2.is_signed_perm()               # R(P)^2 is a Clifford
        r4 = r2 @ r2
        sp = r4.signed_perm_of()
        assert sp is not None and sp[0] == list(range(4 ** n))   # R^4 = diag(+-1)
        assert (r4 @ r4).equals(zmat.ZMat.identity(n))           # R^8 = I


@pytest.mark.parametrize("n", [1, 2, 3])
def test_orthogonality_bounds_and_identity_row(n):
    for seed in range(3):
        tw = seeded_inputs.target_words(n, 6, seed)
        u = zmat.target_from_words(n, tw.paulis, tw.clifford)
        assert u.is_orthogonal()
        assert u.T().is_orthogonal()
        # the identity Pauli is fixed: row 0 and column 0 are e_0
        v = u.raise_to(u.e)
        assert int(v.A[0, 0]) == (1 << (u.e // 2) if u.e % 2 == 0 else 0)
        assert all(int(x) == 0 for x in v.A[0, 1:]) and all(int(x) == 0 for x in v.A[1:, 0])
        # bounds from orthogonality of M and of its Galois conjugate sqrt2 -> -sqrt2
        amax = max(abs(int(x)) for x in u.A.flat)
        bmax = max(abs(int(x)) for x in u.B.flat)
        assert amax * amax <= (1 << u.e)
        assert 2 * bmax * bmax <= (1 << u.e)
        # Galois conjugate is orthogonal too
        assert zmat.ZMat(u.A, -u.B, u.e).is_orthogonal()


def test_sparse_structure_of_rotation():
    # exactly 4^n/2 columns hold two entries +-1/sqrt2, the others are unit columns
    for n in (1, 2, 3):
        for p in (1, 4 ** n - 1):
            r = zmat.rot_hat(p, n).raise_to(1)
            two = sum(1 for q in range(4 ** n) if sum(int(v) != 0 for v in r.A[:, q]) == 2)
            assert two == 4 ** n // 2


def test_clifford_words_are_signed_permutations():
    for n in (1, 2, 3):
        d = zmat.clifford_from_word(n, seeded_inputs.random_clifford_word(n, 5))
        sp = d.signed_perm_of()
        assert sp is not None and sp[0][0] == 0 and sp[1][0] == 1


def test_clifford_channel_rep_via_trace_formula():
    n = 2
    word = seeded_inputs.random_clifford_word(n, 9, length=6)
    u = cy.CycMat.identity(n)
    for c in word:
        u = u @ cy.rotation(c, n) @ cy.rotation(c, n)
    assert zmat_from_trace(u, n).equals(zmat.clifford_from_word(n, word))
    # a signed permutation D: D P_q D^dag = sign[q] P_perm[q], checked on explicit matrices
    perm, sign = zmat.clifford_from_word(n, word).signed_perm_of()
    uc = u.to_complex()
    for q in range(16):
        lhs = uc @ pauli.matrix(q, n) @ uc.conj().T
        assert np.allclose(lhs, sign[q] * pauli.matrix(perm[q], n), atol=1e-12)


def test_canonical_form_left_clifford_invariance():
    for n in (1, 2, 3):
        tw = seeded_inputs.target_words(n, 5, 3)
        u = zmat.target_from_words(n, tw.paulis, tw.clifford)
        base = zmat.canonical_form(u)
        for s in range(4):
            d = zmat.clifford_from_word(n, seeded_inputs.random_clifford_word(n, 100 + s))
            assert zmat.canonical_form(d @ u) == base
        # a rotation on the left changes the coset
        assert zmat.canonical_form(zmat.rot_hat(1, n) @ u) != base


def _sign_decimal(a, b):
    """Sign of a + b sqrt2 by 120-digit decimal arithmetic (independent of zmat's exact rule)."""
    import decimal
    with decimal.localcontext() as ctx:
        ctx.prec = 120
        v = decimal.Decimal(a) + decimal.Decimal(b) * decimal.Decimal(2).sqrt()
    return (v > 0) - (v < 0)


def test_real_sign_against_decimal_and_pell_boundary():
    """zmat.real_sign, which decides every row sign of the canonical form, against 120-digit
    decimal arithmetic: random pairs of every sign pattern and size, and the hardest cases, the Pell
    pairs p^2 - 2 q^2 = +-1 whose p - q sqrt2 = +-1 / (p + q sqrt2) is within 1e-40 of zero."""
    rng = np.random.default_rng(17)
    cases = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (3, -2), (-3, 2), (1, -1), (-1, 1), (2, -1), (-2, 1)]
    for bits in (3, 10, 31, 62, 120):
        for _ in range(200):
            a = int(rng.integers(-(1 << 62), 1 << 62)) >> max(0, 62 - bits)
            b = int(rng.integers(-(1 << 62), 1 << 62)) >> max(0, 62 - bits)
            cases.append((a << max(0, bits - 62), b << max(0, bits - 62)))
    p, q = 1, 1                      # 1 + sqrt2 and its powers give every Pell pair
    for _ in range(60):
        cases += [(p, -q), (-p, q)]
        p, q = p + 2 * q, p + q
    assert max(abs(a) for a, _ in cases) > 10 ** 30
    for a, b in cases:
        assert zmat.real_sign(a, b) == _sign_decimal(a, b), (a, b)


def test_canonical_form_row_sign_rule():
    """A row whose first nonzero entry is -3 + 2 sqrt2 (about -0.17, negative although b > 0) is
    negated in the canonical form; one whose first nonzero entry is 3 - 2 sqrt2 is kept; zero entries
    before it do not count; rows then sort as integer tuples."""
    A = np.zeros((16, 16), dtype=object)
    B = np.zeros((16, 16), dtype=object)
    A[0, 0], B[0, 0], A[0, 5] = -3, 2, 7      # row 0: (-3 + 2 sqrt2, ..., 7 at column 5)
    A[1, 1], B[1, 1], A[1, 2] = 3, -2, -1     # row 1: first nonzero at column 1, positive
    A[2, 3], B[2, 4] = 0, -1                  # row 2: first nonzero is -sqrt2 at column 4
    for r in range(3, 16):
        A[r, r] = 1
    e, rows = zmat.canonical_form(zmat.ZMat(A, B, 0))
    row0 = [0] * 32
    row0[0], row0[1], row0[10] = 3, -2, -7
    row1 = [0] * 32
    row1[2], row1[3], row1[4] = 3, -2, -1
    row2 = [0] * 32
    row2[9] = 1
    assert e == 0
    assert tuple(row0) in rows and tuple(row1) in rows and tuple(row2) in rows
    assert list(rows) == sorted(rows)
