"""GPU: the steps around the solve (Sec. 1) through the C ABI: the reduction
H = Q0^T A Q0 (hsrq_gehrd) and the back-transform z = Q0 x (hsrq_ormhr)
against the reference's plain Householder reduction, and the whole chain
A -> H -> eigenvectors of H -> eigenvectors of A."""
import numpy as np
import pytest

from oracle import oracle as O
from tests.parity import EPS, direction, vec
from workloads import generators as g

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def solver():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2101_05063_amd import Solver
    s = Solver(0)
    yield s
    s.close()


def dev(A):
    A = np.asarray(A, dtype=np.float64)
    return torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()


def host(T):
    return T.t().contiguous().cpu().numpy().T.copy()


@pytest.mark.parametrize("n", [3, 64, 300, 1000])
def test_gehrd_and_ormhr_against_reference(solver, n):
    """Reflectors, tau and H against the reference's reduction of the same A
    (summation orders differ, so to a tolerance of 100 n eps ||A||); Q0 from
    the back-transform of the identity orthogonal and Q0^T A Q0 = H on the
    GPU's own results; the back-transform of a random block against the
    reference's."""
    rng = np.random.default_rng(7000 + n)
    A = rng.standard_normal((n, n))
    print(f"[gpu] gehrd n={n}", flush=True)
    Ad = dev(A)
    tau = solver.gehrd(Ad)
    torch.cuda.synchronize()
    Rg, taug = host(Ad), tau.cpu().numpy()
    Ro, tauo = O.hessenberg_reduce(A)
    nA = np.linalg.norm(A)
    tol = 100 * n * EPS * max(1.0, nA)
    assert np.max(np.abs(np.triu(Rg, -1) - np.triu(Ro, -1))) <= tol
    assert np.max(np.abs(np.tril(Rg, -2) - np.tril(Ro, -2))) <= 100 * n * EPS * 10
    assert np.max(np.abs(taug[:n - 1] - tauo[:n - 1])) <= 100 * n * EPS
    Q = host(solver.ormhr(Ad, tau, dev(np.eye(n))))
    torch.cuda.synchronize()
    assert np.max(np.abs(Q.T @ Q - np.eye(n))) <= 20 * n * EPS
    Hg = np.triu(Rg, -1)
    assert np.max(np.abs(Q.T @ A @ Q - Hg)) <= tol
    Z = rng.standard_normal((n, 12))
    Zg = host(solver.ormhr(Ad, tau, dev(Z)))
    torch.cuda.synchronize()
    Zo = O.apply_q(Ro, tauo, Z)
    assert np.max(np.abs(Zg - Zo)) <= 100 * n * EPS * np.abs(Z).max()


def test_eigenvectors_of_a_general_matrix(solver):
    """A (n = 600, random) reduced on the GPU, eigenvectors of its Hessenberg
    form by the solve (real eigenvalues and complex pairs as shifts), mapped
    back by Q0: every converged result is an eigenvector of A within the
    residual bar ||A z - lambda z|| <= 10 n eps ||A||_F ||z||, and matches
    numpy's eigenvector of A in direction for well-separated eigenvalues."""
    rng = np.random.default_rng(7100)
    n = 600
    A = rng.standard_normal((n, n))
    w, V = np.linalg.eig(A)
    sep = np.array([np.min(np.abs(np.delete(w, k) - w[k])) for k in range(n)])
    real = [k for k in range(n) if abs(w[k].imag) == 0][:8]
    cplx = [k for k in range(n) if w[k].imag > 0][:4]
    idx = real + cplx
    wr, wi = w[idx].real.copy(), w[idx].imag.copy()
    Ad = dev(A)
    tau = solver.gehrd(Ad)
    X = dev(np.ones((n, g.ncols(wi))))
    E, mu, info, _ = solver.dhsrq3(Ad, wr, wi, X)  # only the Hessenberg part of Ad is read
    solver.ormhr(Ad, tau, X)
    torch.cuda.synchronize()
    Z, info = host(X), info.cpu().numpy()
    cols, _ = O.columns_of(wi)
    assert np.sum(info == 0) >= len(idx) - 2
    checked = 0
    for l, k in enumerate(idx):
        if info[l] != 0:
            continue
        z = vec(Z, cols, wi, l)
        lam = complex(wr[l], wi[l])
        res = np.linalg.norm(A @ z - lam * z) / (np.linalg.norm(A) * np.linalg.norm(z))
        assert res <= 10 * n * EPS, (l, res)
        if sep[k] >= 1e-3 * np.abs(w).max():
            assert direction(z, V[:, k]) >= 1.0 - 1e-10, (l, 1.0 - direction(z, V[:, k]))
            checked += 1
    assert checked >= 4


@pytest.mark.parametrize("n", [2100, 4500, 8200])
def test_gehrd_large_properties(solver, n):
    """The sizes whose column kernel differs from the small cases' (4 and 8
    rows per thread in registers, and the general kernel past 8192 rows),
    checked by properties that hold at any size, on the GPU in FP64:
    Q0 orthogonal, Q0^T A Q0 = H, and the first reflector equal to the one
    Householder's construction gives for column 0 of A (it depends on that
    column alone: beta = -sign(a) ||x||, tau = (beta - a) / beta, v = x(2:)
    / (a - beta), x = A(1:n, 0), a = x(1))."""
    rng = np.random.default_rng(9000 + n)
    A = rng.standard_normal((n, n))
    print(f"[gpu] gehrd properties n={n}", flush=True)
    Ad = dev(A)
    A_gpu = Ad.clone()
    tau = solver.gehrd(Ad)
    Q = solver.ormhr(Ad, tau, torch.eye(n, dtype=torch.float64, device=Ad.device).t())  # column-major
    torch.cuda.synchronize()
    H = torch.triu(Ad, -1)
    eye = torch.eye(n, dtype=torch.float64, device=Ad.device)
    orth = float((Q.t().contiguous() @ Q - eye).abs().max())
    assert orth <= 20 * n * EPS, orth
    nA = float(torch.linalg.norm(A_gpu))
    sim = float((Q.t().contiguous() @ (A_gpu @ Q) - H).abs().max())
    assert sim <= 100 * n * EPS * nA, (sim, nA)
    x = A[1:, 0]
    a = x[0]
    beta = -np.copysign(np.linalg.norm(x), a)
    R0 = host(Ad[:, :1])[:, 0]
    t0 = float(tau[0])
    assert abs(R0[0] - A[0, 0]) == 0.0
    assert abs(R0[1] - beta) <= 10 * n * EPS * abs(beta)
    assert abs(t0 - (beta - a) / beta) <= 10 * n * EPS
    v = x[1:] / (a - beta)
    assert np.max(np.abs(R0[2:] - v)) <= 10 * n * EPS * max(1.0, np.abs(v).max())
