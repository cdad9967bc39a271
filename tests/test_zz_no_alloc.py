"""GPU: hsrq_dhsrq3_noalloc (the solve for callers that cannot allocate, its
workspace a fixed device array inside the library) through the C ABI against
hsrq_dhsrq3 with a caller workspace: the same kernels on the same inputs, so
the results must agree bit for bit; two calls in a row, the second smaller,
and a problem beyond the array's size refused before anything runs."""
import numpy as np
import pytest

from workloads import generators as g

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(A):
    A = np.asarray(A, dtype=np.float64)
    return torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()


def host(T):
    return T.t().contiguous().cpu().numpy().T.copy()


def problem(seed, n, nreal, ncplx):
    rng = np.random.default_rng(seed)
    H = g.random_hessenberg(n, rng)
    sc = np.abs(np.linalg.eigvals(H)).max()
    wr = np.concatenate([rng.uniform(-sc, sc, nreal), rng.uniform(-sc, sc, ncplx)])
    wi = np.concatenate([np.zeros(nreal), rng.uniform(0.1, 1.0, ncplx) * sc * np.where(rng.random(ncplx) < 0.5, 1, -1)])
    B = rng.standard_normal((n, g.ncols(wi)))
    return H, wr, wi, B


@pytest.mark.parametrize("rotations", [0, 1])
def test_noalloc_equals_workspace_call(rotations):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2101_05063_amd import HSRQ_OK, Solver
    s = Solver(0)
    for k, (n, nr, nc, nb) in enumerate([(700, 9, 3, 64), (150, 3, 1, 0)]):  # the second call smaller
        H, wr, wi, B = problem(9000 + 10 * rotations + k, n, nr, nc)
        print(f"[gpu] noalloc call {k}: n={n} m={len(wr)} nb={nb} rotations={rotations}", flush=True)
        Hd = dev(H)
        X1, X2 = dev(B), dev(B)
        st, E1, mu1, i1, r1 = s.dhsrq3_noalloc(Hd, wr, wi, X1, nb=nb, residual=True, rotations=rotations)
        assert st == HSRQ_OK
        E2, mu2, i2, r2 = s.dhsrq3(Hd, wr, wi, X2, nb=nb, residual=True, rotations=rotations)
        torch.cuda.synchronize()
        assert np.array_equal(host(X1), host(X2)), k
        for a, b in ((E1, E2), (mu1, mu2), (i1, i2), (r1, r2)):
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()), k
        assert np.all(i1.cpu().numpy() <= 1)
    s.close()


def test_noalloc_refuses_a_problem_beyond_the_array():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2101_05063_amd import HSRQ_ERR_TOO_LARGE, NOALLOC_SCRATCH_BYTES, Solver
    s = Solver(0)
    n, m = 2500, 600
    assert s.workspace_size(n, np.zeros(m)) > NOALLOC_SCRATCH_BYTES
    H = g.random_hessenberg(n, 5)
    B = np.ones((n, m))
    X = dev(B)
    st, *_ = s.dhsrq3_noalloc(dev(H), np.linspace(-1, 1, m), np.zeros(m), X)
    assert st == HSRQ_ERR_TOO_LARGE
    torch.cuda.synchronize()
    assert np.array_equal(host(X), B)  # nothing ran
    s.close()
