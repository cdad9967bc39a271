"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no arithmetic of the solver: it only builds Hessenberg
matrices, shift lists and starting vectors.  Both the GPU tests and the
reference use it.

Recipes (seed = 1000 + k for configuration k, numpy ``default_rng``):

* ``random_hessenberg``: entries N(0,1) on and above the diagonal, subdiagonal
  |N(0,1)| + 0.1 (so H is unreduced).
* ``graded``: D H D^-1 with D_ii = 10^(decades * i / n), i = 1..n.
* ``paper_h1``: the first test problem of Sec. 5.2 (quasi-triangular T with
  t_kk = k or 2x2 blocks [[k, k], [-k, k]], strictly upper part U(0,1], a random
  Householder similarity, then the Hessenberg reduction).
* ``paper_h2`` / ``paper_h3``: the "bad" and "good" systems of Sec. 5.2,
  H = R Q2 + gamma I in closed form.
* ``config_c1`` .. ``config_c5_pool``: the five benchmark configurations.
  Shifts are eigenvalues computed in FP64 on the host by LAPACK (scipy), which
  for the large matrices are cached in ``workloads/cache`` by ``make_cache.py``.
"""
from __future__ import annotations

import math
import os

import numpy as np

CACHE_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cache")


# --------------------------------------------------------------------------
# matrices
# --------------------------------------------------------------------------
def random_hessenberg(n, rng):
    """Upper part N(0,1), subdiagonal |N(0,1)| + 0.1 (column-major float64)."""
    if not isinstance(rng, np.random.Generator):
        rng = np.random.default_rng(rng)
    A = rng.standard_normal((n, n))
    H = np.triu(A)
    if n > 1:
        sub = np.abs(rng.standard_normal(n - 1)) + 0.1
        H[np.arange(1, n), np.arange(n - 1)] = sub
    return np.asfortranarray(H)


def graded(H, decades=300.0):
    """D H D^-1 with D_ii = 10^(decades * i / n), i = 1..n (row i scaled up,
    column j scaled down)."""
    n = H.shape[0]
    e = decades * np.arange(1, n + 1) / n
    # scale by exact ratios 10^(e_i - e_j) computed per entry to avoid overflow
    ratio = 10.0 ** (e[:, None] - e[None, :])
    G = np.where(np.tril(np.ones((n, n), dtype=bool), -2), 0.0, H * ratio)
    return np.asfortranarray(G)


def haar_orthogonal(n, rng):
    Z = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    return Q * np.sign(np.diag(R))[None, :]


def paper_h2(n, gamma=2.0):
    """H2 = R2 Q2 + gamma I (Sec. 5.2): r2(i,i) = n-i+1, r2(i,j) = -n for j > i;
    q2(i,j) = -1 for i-1 = j or (i = 1, j = n)."""
    R = np.triu(np.full((n, n), -float(n)), 1) + np.diag(np.arange(n, 0, -1, dtype=float))
    Q = np.zeros((n, n))
    for i in range(n):
        j = (i - 1) % n
        Q[i, j] = -1.0
    return np.asfortranarray(R @ Q + gamma * np.eye(n)), R, Q


def paper_h3(n, gamma=2.0):
    """H3 = R3 Q2 + gamma I: r3(i,i) = n+1-i, r3(i,j) = 1/2 for j > i."""
    R = np.triu(np.full((n, n), 0.5), 1) + np.diag(np.arange(n, 0, -1, dtype=float))
    _, _, Q = paper_h2(n, gamma)
    return np.asfortranarray(R @ Q + gamma * np.eye(n)), R, Q


def _hessenberg(A):
    import scipy.linalg
    H, Qh = scipy.linalg.hessenberg(A, calc_q=True)
    H = np.triu(H, -1)
    return np.asfortranarray(H), Qh


def paper_h1(n, real_fraction=1.0, seed=0):
    """First test problem of Sec. 5.2.  Returns (H, eigenvalues, T, Qtot) with
    H = Qtot^T T Qtot."""
    rng = np.random.default_rng(seed)
    T = np.triu(rng.uniform(0.0, 1.0, (n, n)), 1)
    T[T == 0.0] = 0.5  # U(0,1]
    T = np.triu(T, 1)
    nreal = int(round(real_fraction * n))
    if (n - nreal) % 2:
        nreal += 1
    lam = []
    k = 1
    i = 0
    while i < n:
        if i < nreal:
            T[i, i] = k
            lam.append(complex(k))
            i += 1
        else:
            T[i, i] = k; T[i, i + 1] = k; T[i + 1, i] = -k; T[i + 1, i + 1] = k
            lam.append(complex(k, k))
            lam.append(complex(k, -k))
            i += 2
        k += 1 if i <= nreal else 2
    v = rng.standard_normal(n)
    v /= np.linalg.norm(v)
    Q0 = np.eye(n) - 2.0 * np.outer(v, v)
    A = Q0 @ T @ Q0
    H, Qh = _hessenberg(A)
    return H, np.array(lam), T, (Q0 @ Qh)


# --------------------------------------------------------------------------
# quasi-triangular construction with known eigenvectors (configuration C1)
# --------------------------------------------------------------------------
def quasi_triangular(n, nreal, rng, min_gap=0.05):
    """T with nreal real eigenvalues U[-1,1] (pairwise gap >= min_gap), the rest
    2x2 blocks [[a, b], [-b, a]] (a, b ~ U[-1,1]) in a random block order, and
    strictly upper entries N(0,1)/sqrt(n).  Returns (T, blocks) where blocks is
    a list of (start, size, eigenvalue)."""
    reals = []
    while len(reals) < nreal:
        x = rng.uniform(-1.0, 1.0)
        if all(abs(x - r) >= min_gap for r in reals):
            reals.append(x)
    npair = (n - nreal) // 2
    assert nreal + 2 * npair == n
    kinds = [("r", r) for r in reals] + [("c", None)] * npair
    order = rng.permutation(len(kinds))
    T = np.triu(rng.standard_normal((n, n)) / math.sqrt(n), 1)
    blocks = []
    i = 0
    for o in order:
        kind, val = kinds[o]
        if kind == "r":
            T[i, i] = val
            blocks.append((i, 1, complex(val)))
            i += 1
        else:
            a, b = rng.uniform(-1.0, 1.0, 2)
            T[i, i] = a; T[i, i + 1] = b; T[i + 1, i] = -b; T[i + 1, i + 1] = a
            blocks.append((i, 2, complex(a, abs(b))))
            i += 2
    return T, blocks


def quasi_triangular_eigvec(T, blocks, k):
    """Right eigenvector u of the quasi-triangular T for the 1x1 block at row k
    (block back substitution, u(k) = 1, u(k+1:) = 0)."""
    n = T.shape[0]
    lam = T[k, k]
    u = np.zeros(n)
    u[k] = 1.0
    starts = [b for b in blocks if b[0] < k]
    for (r0, sz, _) in reversed(starts):
        r1 = r0 + sz
        rhs = -T[r0:r1, r1:k + 1] @ u[r1:k + 1]
        u[r0:r1] = np.linalg.solve(T[r0:r1, r0:r1] - lam * np.eye(sz), rhs)
    return u


def config_c1(seed=1001, n=256, nreal=16):
    """Plain method, n=256: 16 real eigenvalues, shifts perturbed by 1e-15
    relative, all-ones starting vectors; also returns the exact eigenvectors
    of H for those eigenvalues (columns of ``V``)."""
    rng = np.random.default_rng(seed)
    T, blocks = quasi_triangular(n, nreal, rng)
    Q = haar_orthogonal(n, rng)
    A = Q @ T @ Q.T
    H, Qh = _hessenberg(A)
    assert np.all(np.diag(H, -1) != 0.0)
    rb = [b for b in blocks if b[1] == 1]
    wr = np.array([b[2].real for b in rb]) * (1.0 + 1e-15)
    wi = np.zeros(len(rb))
    V = np.stack([Qh.T @ (Q @ quasi_triangular_eigvec(T, blocks, b[0])) for b in rb], axis=1)
    V /= np.linalg.norm(V, axis=0)
    B = np.ones((n, len(rb)), order="F")
    return dict(name="c1", H=H, wr=wr, wi=wi, B=B, V=V, exact=np.array([b[2].real for b in rb]))


# --------------------------------------------------------------------------
# shift selection from host eigenvalues
# --------------------------------------------------------------------------
def host_eigvals(H):
    import scipy.linalg
    return scipy.linalg.eigvals(H, check_finite=False, overwrite_a=False)


def separation(ev):
    """Distance of each eigenvalue to the nearest other eigenvalue (the
    conjugate of a complex one included)."""
    ev = np.asarray(ev)
    pts = np.concatenate([ev, np.conj(ev[np.abs(ev.imag) > 0])])
    sep = np.empty(ev.shape[0])
    for i, z in enumerate(ev):
        d = np.abs(pts - z)
        d[i] = np.inf
        if z.imag != 0.0:
            d[np.abs(pts - np.conj(z)) == 0.0] = np.inf
            d[i] = np.inf
            # the conjugate partner of z itself is a distinct eigenvalue
            d_conj = abs(z - np.conj(z))
            d = np.append(d, d_conj)
        sep[i] = d.min()
    return sep


def pick_shifts(ev, nreal, npair, rng=None, prefer_sep=None):
    """nreal real eigenvalues and npair complex ones (Im > 0, one member per
    conjugate pair).  With ``prefer_sep`` the best separated come first.
    Returns (wr, wi, sep)."""
    ev = np.asarray(ev)
    tol = 1e-12 * max(1.0, np.abs(ev).max())
    real = ev[np.abs(ev.imag) <= tol].real
    cplx = ev[ev.imag > tol]
    sep_all = separation(np.concatenate([real + 0j, cplx]))
    sr, sc = sep_all[:real.size], sep_all[real.size:]
    if prefer_sep is not None:
        ir = np.argsort(-sr)[:nreal]
        ic = np.argsort(-sc)[:npair]
    else:
        rng = rng or np.random.default_rng(0)
        ir = rng.permutation(real.size)[:nreal]
        ic = rng.permutation(cplx.size)[:npair]
    wr = np.concatenate([real[ir], cplx[ic].real])
    wi = np.concatenate([np.zeros(ir.size), cplx[ic].imag])
    sep = np.concatenate([sr[ir], sc[ic]])
    return wr, wi, sep


def ncols(wi):
    return int(np.sum(np.where(np.asarray(wi) != 0.0, 2, 1)))


def ones_start(n, wi):
    """All-ones starting vectors in the column layout of the shifts (complex:
    real part ones, imaginary part zero)."""
    B = np.zeros((n, ncols(wi)), order="F")
    c = 0
    for w in wi:
        B[:, c] = 1.0
        c += 2 if w != 0.0 else 1
    return B


def _cache_path(name):
    return os.path.join(CACHE_DIR, name + ".npz")


def _cached_eigs(name, H, key):
    path = _cache_path(name)
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        if str(z["key"]) == key:
            return z["ev"]
    ev = host_eigvals(H)
    os.makedirs(CACHE_DIR, exist_ok=True)
    np.savez(path, ev=ev, key=key)
    return ev


def config_c2(seed=1002, n=2000, nreal=150, npair=25):
    """Plain method on GPU, n=2000: 150 real shifts and 25 complex pairs from
    the host eigenvalues, best separated first; all-ones starts."""
    H = random_hessenberg(n, seed)
    ev = _cached_eigs("c2", H, f"c2-{seed}-{n}")
    wr, wi, sep = pick_shifts(ev, nreal, npair, prefer_sep=True)
    nrm2 = np.linalg.norm(H, 2) if n <= 4000 else None
    return dict(name="c2", H=H, wr=wr, wi=wi, B=ones_start(n, wi), sep=sep, norm2=nrm2)


def config_c3(seed=1003, n=8000, m=1000, decades=300.0, grade=True):
    """Overflow stress, n=8000, m=1000 real shifts: the C2 construction graded
    by D H D^-1, D_ii = 10^(300 i / n); the shifts are real eigenvalues of the
    ungraded H (eigenvalues are similarity invariant)."""
    H0 = random_hessenberg(n, seed)
    ev = _cached_eigs("c3", H0, f"c3-{seed}-{n}")
    wr, wi, sep = pick_shifts(ev, m, 0, prefer_sep=True)
    H = graded(H0, decades) if grade else H0
    return dict(name="c3", H=H, H0=H0, wr=wr, wi=wi, B=ones_start(n, wi), sep=sep)


def c4_sizes(seed=1004, count=512, nmin=64, nmax=2048):
    rng = np.random.default_rng(seed)
    ns = np.round(np.exp(rng.uniform(math.log(nmin), math.log(nmax), count))).astype(int)
    ks = rng.integers(4, 65, count)
    return ns, ks, rng


def config_c4(seed=1004, count=512, nmin=64, nmax=2048, complex_frac=0.3):
    """Batching: ``count`` random Hessenberg matrices, n log-uniform in
    [nmin, nmax], 4-64 shifts each (30% complex pairs) from host eigenvalues."""
    ns, ks, rng = c4_sizes(seed, count, nmin, nmax)
    probs = []
    path = _cache_path(f"c4_{seed}_{count}_{nmin}_{nmax}")
    cache = dict(np.load(path, allow_pickle=False)) if os.path.exists(path) else {}
    dirty = False
    for b in range(count):
        n = int(ns[b])
        H = random_hessenberg(n, rng.integers(1 << 62))
        key = f"ev{b}"
        if key in cache and cache[key].shape[0] == n:
            ev = cache[key]
        else:
            ev = host_eigvals(H)
            cache[key] = ev
            dirty = True
        k = int(min(ks[b], n // 2))
        npair = int(round(complex_frac * k))
        nreal = k - npair
        tol = 1e-12 * max(1.0, np.abs(ev).max())
        avail_r = int(np.sum(np.abs(ev.imag) <= tol))
        avail_c = int(np.sum(ev.imag > tol))
        nreal = min(nreal, avail_r)
        npair = min(k - nreal, avail_c)
        wr, wi, sep = pick_shifts(ev, nreal, npair, prefer_sep=True)
        probs.append(dict(H=H, wr=wr, wi=wi, B=ones_start(n, wi), sep=sep))
    if dirty:
        os.makedirs(CACHE_DIR, exist_ok=True)
        np.savez(path, **cache)
    return probs


def config_c5_pool(seed=1005, count=64, nmin=128, nmax=8192, complex_frac=0.3):
    """Serving pool: ``count`` matrices, n log-uniform in [nmin, nmax]; each
    request draws U{1..n/8} shifts (30% complex) from its matrix's host
    eigenvalues.  Returns a list of dict(H, ev)."""
    rng = np.random.default_rng(seed)
    ns = np.round(np.exp(rng.uniform(math.log(nmin), math.log(nmax), count))).astype(int)
    path = _cache_path(f"c5_{seed}_{count}_{nmin}_{nmax}")
    cache = dict(np.load(path, allow_pickle=False)) if os.path.exists(path) else {}
    dirty = False
    pool = []
    for b in range(count):
        n = int(ns[b])
        H = random_hessenberg(n, rng.integers(1 << 62))
        key = f"ev{b}"
        if key in cache and cache[key].shape[0] == n:
            ev = cache[key]
        else:
            ev = host_eigvals(H)
            cache[key] = ev
            dirty = True
        pool.append(dict(H=H, ev=ev))
    if dirty:
        os.makedirs(CACHE_DIR, exist_ok=True)
        np.savez(path, **cache)
    return pool


def c5_request(pool_entry, rng, complex_frac=0.3):
    """One serving request on a pool matrix: U{1..n/8} shifts, 30% complex."""
    H, ev = pool_entry["H"], pool_entry["ev"]
    n = H.shape[0]
    k = int(rng.integers(1, max(1, n // 8) + 1))
    npair = int(round(complex_frac * k))
    nreal = k - npair
    tol = 1e-12 * max(1.0, np.abs(ev).max())
    avail_r = int(np.sum(np.abs(ev.imag) <= tol))
    avail_c = int(np.sum(ev.imag > tol))
    nreal = min(nreal, avail_r)
    npair = min(k - nreal, avail_c)
    wr, wi, _ = pick_shifts(ev, nreal, npair, rng=rng)
    return dict(H=H, wr=wr, wi=wi, B=ones_start(n, wi))


def c5_requests(pool, count, seed=1005, complex_frac=0.3):
    """``count`` serving requests drawn like ``c5_request`` (a uniformly chosen
    pool matrix, U{1..n/8} shifts, 30% complex pairs, chosen at random among
    its host eigenvalues), without the separations or starting vectors (the
    starts are all ones).  Returns a list of (pool index, wr, wi)."""
    rng = np.random.default_rng(seed)
    split = []
    for e in pool:
        ev = np.asarray(e["ev"])
        tol = 1e-12 * max(1.0, np.abs(ev).max())
        split.append((ev[np.abs(ev.imag) <= tol].real, ev[ev.imag > tol]))
    out = []
    for _ in range(count):
        b = int(rng.integers(len(pool)))
        n = pool[b]["H"].shape[0]
        real, cplx = split[b]
        k = int(rng.integers(1, max(1, n // 8) + 1))
        npair = int(round(complex_frac * k))
        nreal = min(k - npair, real.size)
        npair = min(k - nreal, cplx.size)
        ir = rng.permutation(real.size)[:nreal]
        ic = rng.permutation(cplx.size)[:npair]
        wr = np.concatenate([real[ir], cplx[ic].real])
        wi = np.concatenate([np.zeros(ir.size), cplx[ic].imag])
        out.append((b, wr, wi))
    return out


def restart_vectors(n, ntries, seed=1007):
    """Starting vectors for inverse iteration with restarts (Sec. 4.2): the
    all-ones vector first, then ntries - 1 orthonormal vectors orthogonal to
    it and to each other (Q of a QR factorisation of [e, G], G seeded
    Gaussian).  n x ntries, column-major."""
    rng = np.random.default_rng(seed)
    A = np.concatenate([np.ones((n, 1)), rng.standard_normal((n, max(ntries - 1, 0)))], axis=1)
    Q, _ = np.linalg.qr(A)
    S = np.asfortranarray(Q[:, :ntries].copy())
    S[:, 0] = 1.0
    return S


def constant_row_sum_hessenberg(n, rng, mu=0.5):
    """A random unreduced Hessenberg matrix whose rows all sum to mu exactly
    (entries rounded to multiples of 2^-12, so that every row sum is exact in
    floating point, and the diagonal set to make them mu): H e = mu e, so
    every left eigenvector of an eigenvalue other than mu is orthogonal to e,
    and inverse iteration from the all-ones vector cannot converge for such a
    shift."""
    H = np.round(random_hessenberg(n, rng) * 4096.0) / 4096.0
    H[np.arange(1, n), np.arange(n - 1)] = np.maximum(H[np.arange(1, n), np.arange(n - 1)], 2.0 ** -12)
    off = np.triu(H, -1) - np.diag(np.diag(H))
    H[np.arange(n), np.arange(n)] = mu - off.sum(axis=1)
    return H
