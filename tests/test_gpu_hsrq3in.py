"""GPU: inverse iteration with restarts (hsrq_hsrq3in, Sec. 4.2 Algorithm 14,
grouping of Algorithm 15) through the C ABI against the reference's driver
fed the same starting vectors."""
import numpy as np
import pytest

from oracle import oracle as O
from tests.parity import compare
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


def run(solver, H, wr, wi, S, **kw):
    print(f"[gpu] hsrq3in n={H.shape[0]} m={len(wr)} tries={S.shape[1]} {kw}", flush=True)
    X, E, mu, info, tries, res = solver.hsrq3in(dev(H), wr, wi, dev(S), **kw)
    torch.cuda.synchronize()
    out = (host(X), E.cpu().numpy(), mu.cpu().numpy(), info.cpu().numpy(), tries.cpu().numpy())
    return out + ((res.cpu().numpy(),) if res is not None else ())


def row_sum_problem(n, seed):
    """Constant row sums, and shifts at eigenvalues away from the row sum whose
    condition number 1 / |v^H u| is below 1e6 (an ill-conditioned eigenvalue
    can show growth from the rounding-level component of e along its left
    eigenvector, and so converge from e after all)."""
    import scipy.linalg as sl
    rng = np.random.default_rng(seed)
    H = g.constant_row_sum_hessenberg(n, rng)
    w, vl, vr = sl.eig(H, left=True, right=True)
    cond = 1.0 / np.abs(np.sum(np.conj(vl) * vr, axis=0))
    far = (np.abs(w - 0.5) > 0.05 * np.abs(w).max()) & (cond < 1e6)
    real = w[far & (np.abs(w.imag) < 1e-12)].real[:10]
    cplx = w[far & (w.imag > 1e-12)][:3]
    wr = np.concatenate([real, cplx.real])
    wi = np.concatenate([np.zeros(len(real)), -cplx.imag * np.array([1, -1, 1])[:len(cplx)]])
    return H, wr, wi


@pytest.mark.parametrize("nb", [64, 128])
def test_restarts_against_reference(solver, nb):
    """Constant row sums: the all-ones start cannot converge for any of these
    shifts (every left eigenvector of an eigenvalue other than the row sum is
    orthogonal to it), the second start does.  Flags, tries and exponents
    equal the reference's, directions within 1e-9."""
    n = 300
    H, wr, wi = row_sum_problem(n, 6100 + nb)
    S = g.restart_vectors(n, 3)
    Yg, Eg, mug, ig, tg, res = run(solver, H, wr, wi, S, nb=nb, residual=True)
    Yo, Eo, muo, io, to = O.hsrq3in(H, wr, wi, S)
    assert list(to) == [1] * len(wr)
    assert np.array_equal(tg, to)
    compare(Yg, Eg, mug, ig, Yo, Eo, muo, io, wi, dir_tol=1e-9, mu_tol=1e-6)
    assert np.all(res[ig == 0] <= 10 * n * 2.0 ** -52)


def test_groups_give_the_same_bits(solver):
    """A workspace that holds only a few columns makes the driver solve the
    shifts in many groups (Algorithm 15): every result is bit-identical to the
    one-group run (the arithmetic of a column does not depend on the others)."""
    n = 300
    H, wr, wi = row_sum_problem(n, 6200)
    S = g.restart_vectors(n, 3)
    one = run(solver, H, wr, wi, S, nb=64)
    from paper_2101_05063_amd import _opts
    import ctypes
    need = ctypes.c_size_t()
    w4 = np.zeros(2)
    solver.lib.hsrq_hsrq3in_workspace_size(solver.h, n, 2, w4.ctypes.data_as(ctypes.c_void_p),
                                           ctypes.byref(_opts(64)), ctypes.byref(need))
    many = run(solver, H, wr, wi, S, nb=64, work_bytes=need.value + 4096)
    for x, y in zip(one, many):
        assert np.array_equal(x, y)


def test_c3_restarts(solver):
    """C3 (n = 8000, m = 1000, graded) with three starts: the shifts that fail
    the first try are solved again; per shift the try, the flag and the
    exponent equal the reference's driver fed the same starts, and the
    directions agree within 1e-6 (the bar of the C3 parity test).  How many
    shifts converge at each try is printed."""
    c = g.config_c3()
    H, wr, wi = c["H"], c["wr"], c["wi"]
    n = H.shape[0]
    S = g.restart_vectors(n, 3)
    Yg, Eg, mug, ig, tg, res = run(solver, H, wr, wi, S, residual=True)
    print(f"[cpu] reference driver for the 1000 C3 shifts", flush=True)
    Yo, Eo, muo, io, to = O.hsrq3in(H, wr, wi, S)
    for t in range(3):
        print(f"[c3 restarts] try {t}: {int(np.sum((tg == t) & (ig == 0)))} converged", flush=True)
    print(f"[c3 restarts] not converged after 3 tries: {int(np.sum(ig == 1))}", flush=True)
    assert np.array_equal(tg, to)
    compare(Yg, Eg, mug, ig, Yo, Eo, muo, io, wi, dir_tol=1e-6, mu_tol=1e-8)
    assert np.all(res[ig == 0] <= 10 * n * 2.0 ** -52)
