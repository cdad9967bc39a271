"""Pins of the CPU reference against what the paper and the mathematics fix.

Every test here runs on the CPU only.  Each is chosen so that a plausible
mistake in the reference (a dropped term, a wrong sign or index, a transposed
operand, a wrong scale exponent) fails at least one of them.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from workloads import generators as g

EPS = 2.0 ** -52
HERE = os.path.dirname(os.path.abspath(__file__))


def direction(y, z):
    """|y^H z| / (||y|| ||z||) (phase invariant)."""
    return abs(np.vdot(y, z)) / (np.linalg.norm(y) * np.linalg.norm(z))


def floor_log2(fr: Fraction) -> int:
    """Exact floor(log2(fr)) of a positive rational."""
    p, q = fr.numerator, fr.denominator
    e = p.bit_length() - q.bit_length()
    # 2^e <= p/q < 2^(e+1) after at most one correction
    if e >= 0:
        if p < (q << e):
            e -= 1
    else:
        if (p << -e) < q:
            e -= 1
    return e


def exact_norm_exponent(x_sq: Fraction):
    """E = floor(log2 ||x||) + 1 and mu = ||x|| / 2^E for ||x||^2 = x_sq."""
    E = floor_log2(x_sq) // 2 + 1
    mu_sq = x_sq / Fraction(2) ** (2 * E)
    mu = math.sqrt(float(mu_sq))
    return E, mu


# ---------------------------------------------------------------------------
# generators pinned to the paper's printed example
# ---------------------------------------------------------------------------
def test_h2_generator_matches_printed_example():
    rows = [list(map(float, ln.split())) for ln in open(os.path.join(HERE, "golden", "h2_minus_gamma_n6.txt"))
            if ln.strip() and not ln.startswith("#")]
    H2, R2, Q2 = g.paper_h2(6)
    assert np.array_equal(H2 - 2.0 * np.eye(6), np.array(rows))
    assert np.array_equal(R2 @ Q2, np.array(rows))


# ---------------------------------------------------------------------------
# brute force on tiny inputs
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 3, 7, 33, 64])
def test_solution_matches_dense_solve(n):
    rng = np.random.default_rng(100 + n)
    H = g.random_hessenberg(n, rng)
    for lam in [0.37, -1.3 + 0.25j, 0.5 - 2.0j]:
        b = rng.standard_normal(n)
        if isinstance(lam, complex):
            b = b + 1j * rng.standard_normal(n)
        r = O.solve1(H, lam, b)
        x = np.linalg.solve(H - lam * np.eye(n), b)
        nx = np.linalg.norm(x)
        cond = np.linalg.cond(H - lam * np.eye(n))
        assert direction(r["y"], x) > 1.0 - 100 * cond * EPS
        ph = np.vdot(r["y"], x) / abs(np.vdot(r["y"], x))
        assert np.allclose(r["y"] * ph, x / nx, atol=100 * cond * EPS)
        assert abs(np.linalg.norm(r["y"]) - 1.0) < 8 * EPS * math.sqrt(n)
        assert abs(r["mu"] * 2.0 ** r["E"] / nx - 1.0) < 100 * cond * EPS
        assert 0.5 <= r["mu"] < 1.0


def test_n1_closed_form():
    H = np.array([[3.0]])
    r = O.solve1(H, 1.0, np.array([5.0]))
    assert r["y"][0] == 1.0 and r["E"] == 2 and r["mu"] == 0.625  # x = 2.5
    r = O.solve1(H, 3.0 + 4.0j, np.array([5.0 + 0j]))
    x = 5.0 / (3.0 - (3.0 + 4.0j))
    assert abs(r["mu"] * 2.0 ** r["E"] - abs(x)) < 4 * EPS * abs(x)


def test_n2_closed_form():
    H = np.array([[1.0, 2.0], [3.0, 4.0]])
    lam = 0.5
    b = np.array([1.0, -1.0])
    r = O.solve1(H, lam, b, record=True)
    # (H - lam I) = [[0.5, 2], [3, 3.5]], det = -4.25, inverse by cofactors
    x = np.array([3.5 * 1.0 - 2.0 * -1.0, -3.0 * 1.0 + 0.5 * -1.0]) / -4.25
    nx = np.linalg.norm(x)
    assert direction(r["y"], x) > 1 - 1e-15
    # single rotation: a = 3, v = 3.5 -> r = hypot(3, 3.5), c = 3.5/r, s = -3/r
    rr = math.sqrt(3.0 ** 2 + 3.5 ** 2)
    assert abs(r["phi"][1] - rr) <= 2 * EPS * rr
    assert abs(r["c"][1].real - 3.5 / rr) <= 2 * EPS and abs(r["s"][1] + 3.0 / rr) <= 2 * EPS
    assert abs(r["mu"] * 2.0 ** r["E"] / nx - 1) < 1e-15


# ---------------------------------------------------------------------------
# the paper's "bad" and "good" systems in closed form
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["h2", "h3"])
@pytest.mark.parametrize("n", [6, 50, 300])
def test_closed_form_rotations(which, n):
    """H - 2I = R Q2 with Q2 a signed cyclic shift: with the convention
    c = v/r, s = -a/r every rotation is exactly (c, s) = (0, 1), R(k,k) is the
    k-th diagonal of R for k >= 2 and R(1,1) = -n (Sec. 5.2)."""
    H, R, _ = (g.paper_h2 if which == "h2" else g.paper_h3)(n)
    H0 = H.copy()
    bnds = [n, n // 2, 3]
    r = O.solve1(H, 2.0, np.ones(n), record=True, snapshots=bnds)
    assert np.array_equal(H, H0)  # H is not modified
    assert np.all(r["c"][1:] == 0.0)
    assert np.all(r["s"][1:] == 1.0)
    assert np.array_equal(r["phi"][1:], np.diag(R)[1:])
    # with (c, s) = (0, 1) the working column never changes: it stays the
    # shifted last column of H - 2I
    v0 = (H - 2.0 * np.eye(n))[:, n - 1]
    for b in bnds:
        assert np.array_equal(r["snap"][b], v0[:b])


def test_h2_last_pivot():
    for n in [6, 50, 300]:
        H, _, _ = g.paper_h2(n)
        r = O.solve1(H, 2.0, np.ones(n), record=True)
        assert r["phi"][0] == -float(n)


def _exact_rq_solution(R, Q):
    """x with (R Q) x = e, exactly: R y = e by back substitution in rationals,
    x = Q^T y (Q is a signed permutation)."""
    n = R.shape[0]
    Rf = [[Fraction(R[i, j]) for j in range(n)] for i in range(n)]
    y = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        acc = Fraction(1)
        for j in range(i + 1, n):
            if Rf[i][j] != 0:
                acc -= Rf[i][j] * y[j]
        y[i] = acc / Rf[i][i]
    QT = Q.T
    x = [sum(Fraction(QT[i, j]) * y[j] for j in range(n) if QT[i, j] != 0) for i in range(n)]
    return x


def _h2_exact_y(n):
    """R2 y = e exactly in O(n) rational operations: y_i = (1 + n S_i) /
    (n - i + 1), S_i = sum_{j > i} y_j."""
    y = [Fraction(0)] * n
    S = Fraction(0)
    for i in range(n - 1, -1, -1):
        y[i] = (1 + n * S) / (n - i)
        S += y[i]
    return y


@pytest.mark.parametrize("n", [6, 40])
def test_h3_solution_exact(n):
    H, R, Q = g.paper_h3(n)
    x = _exact_rq_solution(R, Q)
    nsq = sum(v * v for v in x)
    E, mu = exact_norm_exponent(nsq)
    r = O.solve1(H, 2.0, np.ones(n))
    xf = np.array([float(v) for v in x])
    assert direction(r["y"], xf) > 1 - 1e-14
    assert r["E"] == E
    assert abs(r["mu"] - mu) < 1e-13


@pytest.mark.parametrize("n", [6, 100, 600, 1200])
def test_h2_scale_exponent_exact(n):
    """The solution of the bad system grows like e^(1.385 n) and leaves the
    double range near n = 512; the reference must still return the exact
    binary exponent of ||x||_2 and the normalised direction."""
    H, R, Q = g.paper_h2(n)
    y = _h2_exact_y(n)
    nsq = sum(v * v for v in y)  # Q2 is orthogonal: ||x|| = ||y||
    E, mu = exact_norm_exponent(nsq)
    r = O.solve1(H, 2.0, np.ones(n))
    assert np.all(np.isfinite(r["y"]))
    assert r["E"] == E
    assert abs(r["mu"] - mu) < 1e-12
    # direction: x = Q2^T y, normalised exactly then rounded
    scale = Fraction(2) ** E
    yn = np.array([float(v / scale) for v in y]) / mu
    xn = Q.T @ yn
    assert direction(r["y"], xn) > 1 - 1e-13
    if n >= 600:
        assert E > 1024  # beyond the double range: scaling was exercised


# ---------------------------------------------------------------------------
# eigenvectors: known by construction and brute force
# ---------------------------------------------------------------------------
def test_c1_known_eigenvectors():
    c = g.config_c1()
    Y, E, mu, info = O.batch(c["H"], c["wr"], c["wi"], c["B"])
    n = c["H"].shape[0]
    res = O.residual(c["H"], c["wr"], c["wi"], Y)
    assert np.all(info == O.OK), info
    assert np.all(res <= 10 * n * EPS), res.max()
    for l in range(Y.shape[1]):
        assert direction(Y[:, l], c["V"][:, l]) >= 1 - 1e-10


def test_paper_h1_eigenvectors():
    n = 40
    H, lam, T, Qt = g.paper_h1(n, real_fraction=0.5, seed=3)
    # one member per pair (Im >= 0)
    sel = lam[lam.imag >= 0]
    wr, wi = sel.real.copy(), sel.imag.copy()
    B = g.ones_start(n, wi)
    Y, E, mu, info = O.batch(H, wr, wi, B)
    res = O.residual(H, wr, wi, Y)
    assert np.all(info == O.OK)
    assert np.all(res <= 10 * n * EPS), res.max()
    w, V = np.linalg.eig(H)
    cols, _ = O.columns_of(wi)
    for l, z in enumerate(sel):
        k = np.argmin(np.abs(w - z))
        y = Y[:, cols[l]] + (1j * Y[:, cols[l] + 1] if wi[l] != 0 else 0)
        assert direction(y, V[:, k]) > 1 - 1e-9


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_brute_force_eig(seed):
    n = 48
    rng = np.random.default_rng(seed)
    H = g.random_hessenberg(n, rng)
    w, V = np.linalg.eig(H)
    sep = g.separation(w)
    nh = np.linalg.norm(H, 2)
    for k in np.argsort(-sep)[:12]:
        z = w[k]
        if z.imag < 0:
            continue
        b = np.ones(n) + 0j
        r = O.solve1(H, z, b)
        assert r["info"] == O.OK
        assert direction(r["y"], V[:, k]) > 1 - 1e-10 * max(1.0, nh / sep[k])
        wr, wi = np.array([z.real]), np.array([z.imag])
        Y = np.stack([r["y"].real, r["y"].imag], axis=1) if z.imag != 0 else r["y"].real[:, None]
        assert O.residual(H, wr, wi, Y)[0] <= 10 * n * EPS


# ---------------------------------------------------------------------------
# invariants and special cases
# ---------------------------------------------------------------------------
def test_rotation_invariants():
    n = 80
    rng = np.random.default_rng(7)
    H = g.random_hessenberg(n, rng)
    for lam in [0.3, 0.3 + 0.4j]:
        r = O.solve1(H, lam, np.ones(n) + 0j, record=True)
        c, s, phi = r["c"][1:], r["s"][1:], r["phi"][1:]
        assert np.all(np.abs(np.abs(c) ** 2 + s ** 2 - 1.0) < 4 * EPS)
        a = np.abs(np.diag(H, -1))
        assert np.all(phi >= a * (1 - 2 * EPS))
        assert np.all(phi > 0)
        assert r["c"][0] == 1.0 and r["s"][0] == 0.0


def test_conjugate_equivariance_bitwise():
    n = 60
    rng = np.random.default_rng(11)
    H = g.random_hessenberg(n, rng)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    lam = -0.4 + 0.9j
    r1 = O.solve1(H, lam, b, record=True)
    r2 = O.solve1(H, np.conj(lam), np.conj(b), record=True)
    assert np.array_equal(r2["y"], np.conj(r1["y"]))
    assert r1["E"] == r2["E"] and r1["mu"] == r2["mu"]
    assert np.array_equal(r2["c"], np.conj(r1["c"]))
    assert np.array_equal(r2["s"], r1["s"])


def test_exactly_singular_shift():
    # H - I = [[-1, 1], [1, -1]]: the rotation gives c = s exactly, so R(1,1) = 0
    H = np.array([[0.0, 1.0], [1.0, 0.0]])
    r = O.solve1(H, 1.0, np.array([1.0, 0.0]), record=True)
    assert r["phi"][0] == 0.0
    assert r["info"] == O.SINGULAR
    assert r["E"] == 2 ** 31 - 1
    assert direction(r["y"], np.array([1.0, 1.0])) > 1 - 1e-15  # null vector of H - I


def test_input_checks():
    H = np.triu(np.ones((5, 5)), -1)
    H[3, 2] = 0.0
    r = O.solve1(H, 0.1, np.ones(5))
    assert r["info"] == O.REDUCED
    H = g.random_hessenberg(5, 1)
    H[1, 3] = np.nan
    assert O.solve1(H, 0.1, np.ones(5))["info"] == O.NONFINITE


def test_far_shift_not_converged():
    n = 64
    H = g.random_hessenberg(n, 5)
    nh = np.linalg.norm(H, 2)
    r = O.solve1(H, 10.0 * nh, np.ones(n))
    assert r["info"] == O.NOT_CONVERGED


def test_batch_equals_single():
    n = 30
    rng = np.random.default_rng(4)
    H = g.random_hessenberg(n, rng)
    wr = np.array([0.1, -0.5, 0.7])
    wi = np.array([0.0, 0.3, 0.0])
    B = rng.standard_normal((n, 4))
    Y, E, mu, info = O.batch(H, wr, wi, B, nthreads=3)
    r0 = O.solve1(H, 0.1, B[:, 0])
    r1 = O.solve1(H, -0.5 + 0.3j, B[:, 1] + 1j * B[:, 2])
    r2 = O.solve1(H, 0.7, B[:, 3])
    assert np.array_equal(Y[:, 0], r0["y"])
    assert np.array_equal(Y[:, 1] + 1j * Y[:, 2], r1["y"])
    assert np.array_equal(Y[:, 3], r2["y"])
    assert list(E) == [r0["E"], r1["E"], r2["E"]]


def test_residual_helper_against_numpy():
    n = 20
    rng = np.random.default_rng(9)
    H = g.random_hessenberg(n, rng)
    Y = rng.standard_normal((n, 3))
    wr = np.array([0.2, 1.0])
    wi = np.array([0.0, 0.5])
    res = O.residual(H, wr, wi, Y)
    y0 = Y[:, 0]
    r0 = np.linalg.norm(H @ y0 - 0.2 * y0) / (np.linalg.norm(H, "fro") * np.linalg.norm(y0))
    y1 = Y[:, 1] + 1j * Y[:, 2]
    r1 = np.linalg.norm(H @ y1 - (1.0 + 0.5j) * y1) / (np.linalg.norm(H, "fro") * np.linalg.norm(y1))
    assert abs(res[0] - r0) < 1e-14 * r0 and abs(res[1] - r1) < 1e-14 * r1


def test_graded_overflow_is_scaled():
    """A reverse-graded matrix makes the unscaled solve overflow; the scaled
    solve stays finite and its direction matches the dense solve of the
    equivalent well-scaled system (eigenvectors map through D)."""
    n = 200
    H0 = g.random_hessenberg(n, 21)
    Hg = g.graded(H0, -300.0)
    w = np.linalg.eigvals(H0)
    z = w[np.argmin(np.abs(w.imag) + (np.abs(w.imag) > 1e-12) * 1e9)].real
    r = O.solve1(Hg, z, np.ones(n))
    assert np.all(np.isfinite(r["y"]))
    assert r["E"] > 1024  # ||x_true|| is beyond the double range
    assert r["info"] in (O.OK, O.NOT_CONVERGED)
    res = O.residual(Hg, np.array([z]), np.array([0.0]), r["y"][:, None])
    assert res[0] <= 10 * n * EPS


# ---------------------------------------------------------------------------
# ||H||_inf and the convergence test of Sec. 4.2, pinned by hand and by exact
# rational arithmetic on both sides of the threshold
# ---------------------------------------------------------------------------
def test_hnorm_inf_hand_computed():
    """||H||_inf is the largest row sum of |h(i,j)| over the Hessenberg part
    (Sec. 4.2 uses it in the convergence test).  The entries below the
    subdiagonal are not part of H and must be ignored; the column sums and the
    full-matrix row sums give different values, so an oracle that took the
    1-norm or read the whole array fails."""
    H = np.array([[1.0, -2.0, 0.5, 3.0],
                  [4.0, 1.0, -1.0, 0.0],
                  [9.0, -0.25, 2.0, -6.0],
                  [7.0, 5.0, 0.5, 1.0]])
    # Hessenberg row sums: 6.5, 6, 0.25 + 2 + 6 = 8.25, 0.5 + 1 = 1.5
    assert O.hnorm_inf(H) == 8.25
    # the alternatives it must not be: Hessenberg column sums 5, 3.25, 4, 10;
    # full-matrix row sums 6.5, 6, 17.25, 13.5
    assert O.hnorm_inf(H.T.copy()) != 8.25


def _exact_hessenberg_solve(H, lam, b):
    """(H - lam I) x = b in exact rational arithmetic, reading only the
    Hessenberg part of H (Gaussian elimination, no pivoting needed: the
    systems used here have a nonzero leading pivot after the row swaps of
    partial pivoting, which is done exactly)."""
    n = H.shape[0]
    A = [[Fraction(float(H[i, j])) if j >= i - 1 else Fraction(0) for j in range(n)] for i in range(n)]
    for i in range(n):
        A[i][i] -= Fraction(float(lam))
    x = [Fraction(float(v)) for v in b]
    for k in range(n):
        p = max(range(k, n), key=lambda r: abs(A[r][k]))
        A[k], A[p] = A[p], A[k]
        x[k], x[p] = x[p], x[k]
        for r in range(k + 1, n):
            f = A[r][k] / A[k][k]
            if f:
                for j in range(k, n):
                    A[r][j] -= f * A[k][j]
                x[r] -= f * x[k]
    for k in range(n - 1, -1, -1):
        x[k] = (x[k] - sum(A[k][j] * x[j] for j in range(k + 1, n))) / A[k][k]
    return x


def threshold_system(k):
    """A 3 x 3 unreduced Hessenberg matrix whose solve is nearly exact in
    floating point: h(3,3) equals the shift and h(2,3) = 0, so both rotations
    are (c, s) = (0, -1), R(1,1) = delta = h(1,3) = k 2^-52 and the solution
    is (-4/3, 0, 7 / (3 delta)); the entry below the subdiagonal (100) is not
    part of H.  ||H||_inf = 7 (row 2),
    ||H||_1 = 6.5, ||H||_F = sqrt(32.5 + delta^2); b = (3, 4, 0) has
    ||b||_2 = 5, ||b||_inf = 4, ||b||_1 = 7."""
    delta = k * 2.0 ** -52
    H = np.array([[1.0, -2.0, delta],
                  [-3.0, 4.0, 0.0],
                  [100.0, 0.5, 1.5]])
    return H, 1.5, np.array([3.0, 4.0, 0.0])


def test_convergence_threshold_both_sides():
    """Converged iff ||x_true||_2 / ||b||_2 >= 1 / (10 n eps ||H||_inf) with
    eps = 2^-52 (Sec. 4.2 with the starting vector's norm made explicit).
    The exact solution (rational arithmetic) places the ratio 1% above the
    threshold for one delta and 1% below it for another; the reference must
    flag the first converged and the second not.  Each plausible misreading
    (1-norm or Frobenius norm of H, entries below the subdiagonal counted,
    n instead of 10 n, eps = 2^-53, another norm of b) moves the threshold by
    more than 1% and misclassifies one of the two cases, which the test also
    checks against the exact ratios."""
    n = 3
    eps = Fraction(1, 2 ** 52)

    def ratio_sq(k):
        H, lam, b = threshold_system(k)
        x = _exact_hessenberg_solve(H, lam, b)
        return sum(v * v for v in x) / sum(Fraction(float(v)) ** 2 for v in b)

    T_sq = 1 / (10 * n * eps * 7) ** 2
    # the ratio falls as delta = k 2^-52 grows; the boundary lies near
    # k = 7 / 15 * 210 = 98
    k_lo = max(k for k in range(50, 200) if ratio_sq(k) >= Fraction(101, 100) ** 2 * T_sq)
    k_hi = min(k for k in range(50, 200) if ratio_sq(k) <= Fraction(99, 100) ** 2 * T_sq)
    assert k_lo < k_hi <= k_lo + 6
    for k, want in ((k_lo, O.OK), (k_hi, O.NOT_CONVERGED)):
        H, lam, b = threshold_system(k)
        r = O.solve1(H, lam, b)
        assert r["info"] == want, (k, r["info"])
        x = np.array([float(v) for v in _exact_hessenberg_solve(H, lam, b)])
        assert abs(r["mu"] * 2.0 ** r["E"] / np.linalg.norm(x) - 1.0) < 1e-14
        assert direction(r["y"], x) > 1.0 - 1e-15
    # sensitivity: each misreading's threshold classifies one case wrongly
    nb2, nbi, nb1 = Fraction(25), Fraction(16), Fraction(49)
    wrong = {
        "1-norm of H": (Fraction(13, 2), 10 * n, eps, nb2),
        "Frobenius norm of H": (Fraction(5.70087712549569), 10 * n, eps, nb2),
        "entries below the subdiagonal": (Fraction(102), 10 * n, eps, nb2),
        "n instead of 10 n": (Fraction(7), n, eps, nb2),
        "eps = 2^-53": (Fraction(7), 10 * n, eps / 2, nb2),
        "max-norm of b": (Fraction(7), 10 * n, eps, nbi),
        "1-norm of b": (Fraction(7), 10 * n, eps, nb1),
    }
    for what, (hn, nn, ee, bb) in wrong.items():
        t_sq = 1 / (nn * ee * hn) ** 2
        conv = [ratio_sq(k) * nb2 / bb >= t_sq for k in (k_lo, k_hi)]
        assert conv != [True, False], what


# ---------------------------------------------------------------------------
# inverse iteration with restarts (Sec. 4.2, Algorithm 14)
# ---------------------------------------------------------------------------
def test_restart_closed_form_2x2():
    """H = [[3, 1], [1, 3]] has the eigenvector e = (1, 1) for 4 and (1, -1)
    for 2.  With the shift 2 + 2^-49, the all-ones start gives
    x = e / (2 - 2^-49): no growth, not converged.  The second start
    (1, -1)/sqrt(2), orthogonal to the first, gives x = -(1, -1) 2^49 / sqrt(2):
    ||x|| / ||b|| = 2^49 > 1 / (10 n eps ||H||_inf) = 2^52 / 80, converged on
    the second try, with the eigenvector (1, -1).  The norm itself is only
    determined to about eps ||H|| / sigma_min = 2^-52 * 4 / 2^-49 relative:
    R(1,1) is a difference of terms of size 1/sqrt(2) that cancel down to
    about 2^-49 sqrt(2), so it is checked to 25%."""
    H = np.array([[3.0, 1.0], [1.0, 3.0]])
    lam = 2.0 + 2.0 ** -49
    S = np.array([[1.0, 2 ** -0.5], [1.0, -2 ** -0.5]])
    Y, E, mu, info, tries = O.hsrq3in(H, np.array([lam]), np.array([0.0]), S)
    assert list(tries) == [1] and list(info) == [O.OK]
    assert direction(Y[:, 0], np.array([1.0, -1.0])) > 1.0 - 1e-15
    assert abs(mu[0] * 2.0 ** E[0] / 2.0 ** 49 - 1.0) <= 0.25
    # one try only: the first start's result, flagged not converged
    Y1, E1, mu1, info1, tries1 = O.hsrq3in(H, np.array([lam]), np.array([0.0]), S, ntries=1)
    assert list(tries1) == [0] and list(info1) == [O.NOT_CONVERGED]
    assert direction(Y1[:, 0], np.array([1.0, 1.0])) > 1.0 - 1e-15


def test_restart_constant_row_sums():
    """Rows of H summing to mu make e a right eigenvector, so every left
    eigenvector of another eigenvalue is orthogonal to e and the all-ones
    start cannot converge for those shifts; a start orthogonal to e does.
    Real and complex eigenvalue shifts: all fail the first try and converge on
    the second, to the eigenvectors numpy computes; the restart results equal
    plain solves from the second start."""
    n = 14
    rng = np.random.default_rng(77)
    H = g.constant_row_sum_hessenberg(n, rng)
    assert np.allclose(H @ np.ones(n), 0.5)
    import scipy.linalg as sl
    w, vl, V = sl.eig(H, left=True, right=True)
    cond = 1.0 / np.abs(np.sum(np.conj(vl) * V, axis=0))  # eigenvalue condition numbers
    far = (np.abs(w - 0.5) > 0.1) & (cond < 1e6)
    real = np.where(far & (np.abs(w.imag) < 1e-12))[0][:3]
    cplx = np.where(far & (w.imag > 1e-12))[0][:2]
    wr = np.concatenate([w[real].real, w[cplx].real])
    wi = np.concatenate([np.zeros(len(real)), w[cplx].imag])
    S = g.restart_vectors(n, 3, seed=5)
    assert abs(S[:, 1] @ np.ones(n)) < 1e-13 and abs(S[:, 2] @ S[:, 1]) < 1e-13
    Y, E, mu, info, tries = O.hsrq3in(H, wr, wi, S)
    assert list(tries) == [1] * len(wr) and list(info) == [O.OK] * len(wr)
    cols, _ = O.columns_of(wi)
    for k, idx in enumerate(list(real) + list(cplx)):
        y = Y[:, cols[k]] + (1j * Y[:, cols[k] + 1] if wi[k] else 0)
        assert direction(y, V[:, idx]) > 1.0 - 1e-10
        r = O.solve1(H, complex(wr[k], wi[k]), S[:, 1].astype(complex) if wi[k] else S[:, 1])
        assert np.array_equal(y, r["y"]) and E[k] == r["E"] and mu[k] == r["mu"]


# ---------------------------------------------------------------------------
# the steps around the solve (Sec. 1): Hessenberg reduction and back-transform
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 3, 8, 60, 150])
def test_hessenberg_reduction_against_lapack(n):
    """The reference's reduction against scipy's (LAPACK DGEHRD, the same
    reflector convention): the same H and Q0 to rounding; Q0 orthogonal,
    Q0^T A Q0 = H, H upper Hessenberg, and the eigenvalues kept."""
    import scipy.linalg as sl
    rng = np.random.default_rng(300 + n)
    A = rng.standard_normal((n, n))
    R, tau = O.hessenberg_reduce(A)
    H = O.hessenberg_part(R)
    Q = O.apply_q(R, tau, np.eye(n))
    Hs, Qs = sl.hessenberg(A, calc_q=True)
    tol = 50 * n * EPS * max(1.0, np.linalg.norm(A))
    assert np.max(np.abs(H - Hs)) <= tol
    assert np.max(np.abs(Q - Qs)) <= 50 * n * EPS
    assert np.max(np.abs(Q.T @ Q - np.eye(n))) <= 10 * n * EPS
    assert np.max(np.abs(Q.T @ A @ Q - H)) <= tol
    assert np.all(np.tril(H, -2) == 0.0)
    if n > 2:
        assert tau[n - 2] == 0.0


def test_back_transform_gives_eigenvectors_of_a():
    """Eigenvectors of H mapped by Q0 are eigenvectors of A (z = Q0 x, Sec. 1):
    the reference's solve on H, then apply_q, against numpy's eigenvectors of
    A for well-separated real eigenvalues."""
    rng = np.random.default_rng(5)
    n = 40
    A = rng.standard_normal((n, n))
    R, tau = O.hessenberg_reduce(A)
    H = O.hessenberg_part(R)
    w, V = np.linalg.eig(A)
    real = [k for k in range(n) if abs(w[k].imag) < 1e-12
            and np.min(np.abs(np.delete(w, k) - w[k])) > 1e-2 * np.abs(w).max()][:4]
    assert real
    for k in real:
        r = O.solve1(H, w[k].real, np.ones(n))
        z = O.apply_q(R, tau, r["y"][:, None])[:, 0]
        assert direction(z, V[:, k].real) > 1.0 - 1e-10
        res = np.linalg.norm(A @ z - w[k].real * z) / (np.linalg.norm(A) * np.linalg.norm(z))
        assert res <= 10 * n * EPS
