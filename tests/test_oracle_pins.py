"""Pins of the FP64 CPU oracle to facts other than itself.

Each test ties an oracle routine to something the paper or the mathematics
fixes: closed forms (n = 1, n = 2, diagonal, Kac-Murdock-Szego matrices),
brute force (Gauss-Jordan), library routines in special cases (numpy solve /
eigvalsh, torch autograd of a dense inverse), invariants (A X = I, X = X^H),
finite differences, and the operation counts of Table 1.
"""
import os

import numpy as np
import pytest

import oracle as O
from paper_1111_4144_amd import inputs as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_hpd(rng, n, complex_=True, shift=0.5):
    return G.random_hpd(rng, 1, n, shift=shift, complex_=complex_)[0]


def _relerr(x, y):
    return np.linalg.norm(x - y) / np.linalg.norm(y)


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("a,b,c", [(4.0, 1 + 2j, 3.0), (2.0, -0.5 + 0.25j, 1.0), (9.0, 3.0, 5.0)])
def test_n2_closed_form(a, b, c):
    """Eqs. (3)-(4), (10)-(11) and Section IV for a 2x2 Hermitian matrix."""
    A = np.array([[a, b], [np.conj(b), c]], dtype=np.complex128)
    r, info = O.chol(A)
    assert info == 0
    det = a * c - abs(b) ** 2
    np.testing.assert_allclose(r, [[np.sqrt(a), b / np.sqrt(a)], [0, np.sqrt(c - abs(b) ** 2 / a)]],
                               rtol=1e-15, atol=0)
    rl, d, info = O.ldl(A)
    assert info == 0
    np.testing.assert_allclose(d, [a, c - abs(b) ** 2 / a], rtol=1e-15)
    np.testing.assert_allclose(rl, [[1, b / a], [0, 1]], rtol=1e-15)
    want = np.array([[c, -b], [-np.conj(b), a]]) / det
    for m in ("chol", "ldl"):
        x, info = O.inv_prop(A, m)
        assert info == 0
        np.testing.assert_allclose(x, want, rtol=1e-14, atol=1e-16)


def test_n1_and_diagonal_exact():
    x, info = O.inv_prop(np.array([[4.0]]))
    assert info == 0 and x[0, 0] == 0.25
    d = np.array([4.0, 16.0, 64.0, 0.25, 1.0])          # exact square roots
    for m in ("chol", "ldl"):
        x, info = O.inv_prop(np.diag(d).astype(np.complex128), m)
        assert info == 0
        assert np.array_equal(x, np.diag(1.0 / d).astype(np.complex128))
        x, _ = O.inv_prop(np.eye(7), m)
        assert np.array_equal(x, np.eye(7))


@pytest.mark.parametrize("n,rho", [(5, 0.5), (12, 0.3 + 0.6j), (200, -0.7 + 0.1j), (64, 0.95)])
def test_kms_closed_form(n, rho):
    """Kac-Murdock-Szego a_ij = rho^(j-i): R, D and X = A^{-1} are known exactly."""
    A = G.kms(n, rho)
    s = 1 - abs(rho) ** 2
    i = np.arange(n)
    p = np.maximum(i[None, :] - i[:, None], 0)
    pw = np.triu(np.asarray(rho, np.complex128) ** p)
    r_want = pw * np.where(i == 0, 1.0, np.sqrt(s))[:, None]
    r, info = O.chol(A)
    assert info == 0
    np.testing.assert_allclose(r, r_want, rtol=1e-12, atol=1e-13)
    rl, d, info = O.ldl(A)
    assert info == 0
    np.testing.assert_allclose(d, np.where(i == 0, 1.0, s), rtol=1e-12)
    np.testing.assert_allclose(rl, pw, rtol=1e-12, atol=1e-13)
    x_want = np.zeros((n, n), np.complex128)
    x_want[i, i] = (1 + abs(rho) ** 2) / s
    x_want[0, 0] = x_want[n - 1, n - 1] = 1 / s
    x_want[i[:-1], i[:-1] + 1] = -rho / s
    x_want[i[:-1] + 1, i[:-1]] = -np.conj(rho) / s
    for m in ("chol", "ldl"):
        x, info = O.inv_prop(A, m)
        assert info == 0
        assert np.abs(x - x_want).max() <= 1e-11 * np.abs(x_want).max()


# ---------------------------------------------------------------------------
# brute force and invariants
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("complex_", [True, False])
def test_gauss_jordan_agreement(rng, n, complex_):
    for _ in range(5):
        A = _rand_hpd(rng, n, complex_)
        kappa = O.kappa2(A.astype(np.complex128))
        xg, info = O.gauss_jordan(A)
        assert info == 0
        for fn in (lambda a: O.inv_prop(a, "chol"), lambda a: O.inv_prop(a, "ldl"),
                   lambda a: O.inv_eqsolve(a, "chol"), lambda a: O.inv_eqsolve(a, "ldl"),
                   O.inv_tri):
            x, info = fn(A)
            assert info == 0
            assert _relerr(x, xg) <= 1e-13 * kappa


@pytest.mark.parametrize("n", [7, 16, 33])
def test_invariants_and_cross_methods(rng, n):
    A = _rand_hpd(rng, n, True, shift=0.1)
    x, info = O.inv_prop(A)
    assert info == 0
    assert np.array_equal(x, np.conj(x.T))                 # X = X^H bitwise
    assert np.all(np.diag(x).real > 0)
    kappa = O.kappa2(A)
    assert np.linalg.norm(A @ x - np.eye(n)) <= 1e-14 * n * kappa
    for other in (O.inv_prop(A, "ldl")[0], O.inv_eqsolve(A)[0], O.inv_eqsolve(A, "ldl")[0],
                  O.inv_tri(A)[0]):
        assert _relerr(other, x) <= 1e-14 * kappa


def test_only_upper_triangle_is_read(rng):
    A = _rand_hpd(rng, 9, True)
    P = A.copy()
    P[np.tril_indices(9, -1)] = np.nan
    P[np.diag_indices(9)] += 5j                              # imaginary diagonal ignored
    for m in ("chol", "ldl"):
        assert np.array_equal(O.inv_prop(A, m)[0], O.inv_prop(P, m)[0])


def test_batched_and_varlen_match_single(rng):
    A = G.random_hpd(rng, 6, 5)
    xb, info = O.inv_prop(A)
    assert np.all(info == 0)
    for k in range(6):
        assert np.array_equal(xb[k], O.inv_prop(A[k])[0])
    packed, sizes, offs = G.varlen_spd(40, seed=7)
    x, info = O.inv_prop_varlen(packed, sizes, offs)
    assert np.all(info == 0)
    for b in (0, 17, 39):
        n = sizes[b]
        a = packed[offs[b]:offs[b] + n * n].reshape(n, n)
        assert np.array_equal(x[offs[b]:offs[b] + n * n].reshape(n, n), O.inv_prop(a)[0])


# ---------------------------------------------------------------------------
# factorisations and solves
# ---------------------------------------------------------------------------
def test_factors_reconstruct_and_relate(rng):
    A = _rand_hpd(rng, 10, True)
    r, info = O.chol(A)
    assert info == 0
    assert np.allclose(np.conj(r.T) @ r, A, rtol=0, atol=1e-13 * np.abs(A).max())
    assert np.array_equal(np.tril(r, -1), np.zeros_like(r))
    rl, d, info = O.ldl(A)
    assert info == 0
    assert np.allclose(np.conj(rl.T) @ np.diag(d) @ rl, A, atol=1e-13 * np.abs(A).max())
    # R_chol = diag(sqrt(d)) R_ldl
    assert np.allclose(r, np.sqrt(d)[:, None] * rl, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("complex_", [True, False])
def test_solves_match_library(rng, complex_):
    A = _rand_hpd(rng, 12, complex_)
    y = rng.standard_normal(12) + (1j * rng.standard_normal(12) if complex_ else 0)
    want = np.linalg.solve(A, y)
    r, _ = O.chol(A)
    np.testing.assert_allclose(O.chol_solve(r, y), want, rtol=1e-11)
    rl, d, _ = O.ldl(A)
    np.testing.assert_allclose(O.ldl_solve(rl, d, y), want, rtol=1e-11)


def test_failure_info_and_nan_fill():
    A = np.diag([1.0, -1.0, 2.0]).astype(np.complex128)
    for m in ("chol", "ldl"):
        x, info = O.inv_prop(A, m)
        assert info == 2 and np.all(np.isnan(x.real)) and np.all(np.isnan(x.imag))
    B = np.eye(4, dtype=np.complex128)
    B[1, 3] = np.nan
    assert O.inv_prop(B)[1] == 4                             # NaN reaches pivot 4 first
    assert O.chol(np.zeros((3, 3)))[1] == 1
    # ldl_factor without positivity: an indefinite but non-singular matrix factors
    _, d, info = O.ldl(np.diag([1.0, -2.0, 3.0]), require_pos=False)
    assert info == 0 and np.array_equal(d, [1.0, -2.0, 3.0])


def test_nonhermitian_inverse(rng):
    D = rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6))
    dinv, info = O.inv_nonherm(D)
    assert info == 0
    np.testing.assert_allclose(dinv, np.linalg.inv(D), rtol=1e-10, atol=1e-12)


# ---------------------------------------------------------------------------
# gradient and Newton-Schulz
# ---------------------------------------------------------------------------
def _herm_directions(n, rng):
    dirs = []
    for i in range(n):
        e = np.zeros((n, n), np.complex128)
        e[i, i] = 1
        dirs.append(e)
    for (i, j) in [(0, 1), (1, 3), (2, n - 1)]:
        e = np.zeros((n, n), np.complex128)
        e[i, j] = e[j, i] = 1 / np.sqrt(2)
        dirs.append(e)
        e = np.zeros((n, n), np.complex128)
        e[i, j], e[j, i] = 1j / np.sqrt(2), -1j / np.sqrt(2)
        dirs.append(e)
    z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    z = z + np.conj(z.T)
    dirs.append(z / np.linalg.norm(z))
    return dirs


def test_grad_finite_differences(rng):
    n = 6
    A = _rand_hpd(rng, n, True, shift=1.0)
    Gm = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    x, _ = O.inv_prop(A)
    ga = O.grad(x, Gm)
    assert np.allclose(ga, np.conj(ga.T), atol=1e-14)

    def loss(a):
        return float(np.real(np.sum(np.conj(Gm) * O.inv_prop(a)[0])))

    h = 1e-6
    for e in _herm_directions(n, rng):
        fd = (loss(A + h * e) - loss(A - h * e)) / (2 * h)
        an = float(np.real(np.sum(np.conj(ga) * e)))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


def test_grad_matches_torch_autograd(rng):
    torch = pytest.importorskip("torch")
    n = 5
    A = _rand_hpd(rng, n, True)
    Gm = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    At = torch.tensor(A, dtype=torch.complex128, requires_grad=True)
    X = torch.linalg.inv(At)
    X.backward(torch.tensor(Gm))
    g = At.grad.numpy()
    want = 0.5 * (g + np.conj(g.T))                          # Hermitian projection
    np.testing.assert_allclose(O.grad(O.inv_prop(A)[0], Gm), want, rtol=1e-12, atol=1e-13)


def test_newton_schulz_fixed_point_and_contraction(rng):
    n = 8
    A = _rand_hpd(rng, n, True, shift=1.0)
    xg, _ = O.gauss_jordan(A)
    x1 = O.ns_step(A, xg)
    assert _relerr(x1, xg) <= 1e-14 * O.kappa2(A)
    pert = 1e-5 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    x0 = xg + (pert + np.conj(pert.T)) * np.abs(xg).max()
    e0 = np.linalg.norm(np.eye(n) - A @ x0, 2)
    e1 = np.linalg.norm(np.eye(n) - A @ O.ns_step(A, x0), 2)
    assert e1 <= 1.01 * e0 ** 2 and e1 < e0                 # I - A X1 = (I - A X0)^2


def test_jacobi_eigenvalues_match_library(rng):
    for n in (1, 3, 9, 20):
        A = _rand_hpd(rng, n, True)
        np.testing.assert_allclose(O.herm_eig(A), np.linalg.eigvalsh(A), rtol=1e-11, atol=1e-12)


# ---------------------------------------------------------------------------
# operation counts (Table 1)
# ---------------------------------------------------------------------------
def _counts(n, rng):
    A = _rand_hpd(rng, n, True)
    res = {}
    with O.count_mults() as c:
        O.chol(A)
        res["chol"] = c()
    with O.count_mults() as c:
        O.ldl(A)
        res["ldl"] = c()
    with O.count_mults() as c:
        O.inv_prop(A, "chol")
        res["prop_chol"] = c()
    with O.count_mults() as c:
        O.inv_prop(A, "ldl")
        res["prop_ldl"] = c()
    with O.count_mults() as c:
        O.inv_eqsolve(A)
        res["eqsolve"] = c()
    with O.count_mults() as c:
        O.inv_tri(A)
        res["tri"] = c()
    r, _ = O.chol(A)
    with O.count_mults() as c:
        O.chol_solve(r, np.ones(n, np.complex128))
        res["solve"] = c()
    return res


def _golden():
    vals = {}
    with open(os.path.join(GOLDEN, "table1_operation_counts.txt")) as f:
        for line in f:
            line = line.split("#")[0].split()
            if line:
                num, _, den = line[1].partition("/")
                vals[line[0]] = float(num) / float(den or 1)
    return vals


def test_operation_counts_exact(rng):
    for n in list(range(1, 25)) + [40]:
        c = _counts(n, rng)
        assert c["chol"] == c["ldl"] == (n ** 3 - n) // 6
        assert c["prop_chol"] == c["prop_ldl"] == (n ** 3 - n) // 2
        assert c["eqsolve"] == 5 * (n ** 3 - n) // 6
        assert c["tri"] == (n ** 3 - n) // 2 + n * (n + 1) * (n + 2) // 6
        assert c["solve"] == n * (n - 1)                      # 1/2 n^2 per solve, two solves


def test_operation_counts_table1(rng):
    g = _golden()
    for n in (64, 160, 256):
        c = _counts(n, rng)
        n3 = float(n) ** 3
        assert abs(c["chol"] / n3 - g["decomposition"]) <= 2.0 / n
        assert abs(c["eqsolve"] / n3 - g["equation_solving"]) <= 2.0 / n
        assert abs(c["tri"] / n3 - g["triangular_operations"]) <= 2.0 / n
        assert abs(c["prop_chol"] / n3 - g["proposed"]) <= 2.0 / n
        if n >= 150:
            saving = 100.0 * (c["tri"] - c["prop_chol"]) / n3
            assert g["reduction_percent_low"] <= saving <= g["reduction_percent_high"]
