"""ctypes wrapper of the plain C reference (``hsrq_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may use it; the GPU library never does.

Every function follows the untiled robust RQ solve of the paper (Henry's
sweep, Sec. 2.2 Algorithm 1, with the power-of-two overflow protection of
Sec. 4.1 and the normalisation of Algorithm 11); see the C file header for the
readings of the paper it takes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hsrq_oracle.c")
_LIB = os.path.join(_HERE, "libhsrq_oracle.so")

# info codes (same meaning on both sides, defined independently)
OK, NOT_CONVERGED, SINGULAR, NONFINITE, REDUCED = 0, 1, 2, 3, 4

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fno-finite-math-only",
            "-std=c11", "-shared", "-fPIC", "-pthread", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        d, i, p = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        lib.hsrq_oracle_solve1.argtypes = [i, p, i, d, d, p, p, p, p, p, p,
                                           p, p, p, p, i, p, p, p, p]
        lib.hsrq_oracle_solve1.restype = i
        lib.hsrq_oracle_batch.argtypes = [i, p, i, i, p, p, p, i, p, i, p, p, p, i]
        lib.hsrq_oracle_batch.restype = i
        lib.hsrq_oracle_residual.argtypes = [i, p, i, i, p, p, p, i, p]
        lib.hsrq_oracle_residual.restype = i
        lib.hsrq_oracle_hnorm_inf.argtypes = [i, p, i]
        lib.hsrq_oracle_hnorm_inf.restype = d
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _fortran(H):
    H = np.asarray(H, dtype=np.float64)
    return np.asfortranarray(H)


def columns_of(wi) -> np.ndarray:
    """First column of every shift: one column per real shift, two ([re im])
    per complex shift (Sec. 4.3, interleaved storage)."""
    w = np.where(np.asarray(wi) != 0.0, 2, 1)
    return np.concatenate([[0], np.cumsum(w)[:-1]]).astype(np.int64), int(w.sum())


def solve1(H, lam, b, record=False, snapshots=()):
    """Solve (H - lam I) x = b for one shift.

    Returns dict(y, E, mu, info) and, with ``record``, the rotations
    c (complex), s, phi indexed by column k (0-based; entry 0 is padding with
    phi[0] = Re R(1,1)), and the working-column snapshots for every boundary b
    in ``snapshots`` (the first b entries of v after all rotations with index
    >= b were applied).
    """
    lib = _load()
    H = _fortran(H)
    n = H.shape[0]
    lam = complex(lam)
    b = np.asarray(b)
    cplx = lam.imag != 0.0 or np.iscomplexobj(b)
    bre = np.ascontiguousarray(b.real, dtype=np.float64)
    bim = np.ascontiguousarray(b.imag, dtype=np.float64) if cplx else None
    yre = np.zeros(n)
    yim = np.zeros(n) if cplx else None
    E = np.zeros(1, dtype=np.int32)
    mu = np.zeros(1)
    rc = rci = rs = rp = None
    if record:
        rc, rci, rs, rp = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n)
    snaps = sorted(set(int(s) for s in snapshots), reverse=True)
    sk = np.array(snaps, dtype=np.int32) if snaps else None
    offs = np.concatenate([[0], np.cumsum(snaps)[:-1]]).astype(np.int64) if snaps else None
    tot = int(sum(snaps))
    sre = np.zeros(max(tot, 1)) if snaps else None
    sim = np.zeros(max(tot, 1)) if snaps else None
    info = lib.hsrq_oracle_solve1(n, _ptr(H), n, lam.real, lam.imag, _ptr(bre), _ptr(bim),
                                  _ptr(yre), _ptr(yim), _ptr(E), _ptr(mu),
                                  _ptr(rc), _ptr(rci), _ptr(rs), _ptr(rp),
                                  len(snaps), _ptr(sk), _ptr(offs), _ptr(sre), _ptr(sim))
    out = {"y": yre + 1j * yim if cplx else yre, "E": int(E[0]), "mu": float(mu[0]), "info": int(info)}
    if record:
        out.update(c=rc + 1j * rci, s=rs, phi=rp)
    if snaps:
        out["snap"] = {bnd: sre[o:o + bnd] + 1j * sim[o:o + bnd] if cplx else sre[o:o + bnd].copy()
                       for bnd, o in zip(snaps, offs)}
    return out


def batch(H, wr, wi, B, nthreads=None):
    """All shifts of one matrix, threaded over shifts.

    ``B`` is n x ncols in the caller's layout (one column per real shift, two
    adjacent [re im] columns per complex shift).  Returns (Y, E, mu, info).
    """
    lib = _load()
    H = _fortran(H)
    n = H.shape[0]
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    wi = np.ascontiguousarray(wi, dtype=np.float64)
    m = wr.shape[0]
    B = np.asfortranarray(B, dtype=np.float64)
    Y = np.zeros_like(B, order="F")
    E = np.zeros(m, dtype=np.int32)
    mu = np.zeros(m)
    info = np.zeros(m, dtype=np.int32)
    if nthreads is None:
        # the host share of one GPU is 16 threads, whatever the machine has
        nthreads = min(16, len(os.sched_getaffinity(0)))
    lib.hsrq_oracle_batch(n, _ptr(H), n, m, _ptr(wr), _ptr(wi), _ptr(B), n, _ptr(Y), n,
                          _ptr(E), _ptr(mu), _ptr(info), int(nthreads))
    return Y, E, mu, info


def residual(H, wr, wi, Y):
    """||H y - lambda y||_2 / (||H||_F ||y||_2) per shift, in long double."""
    lib = _load()
    H = _fortran(H)
    n = H.shape[0]
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    wi = np.ascontiguousarray(wi, dtype=np.float64)
    Y = np.asfortranarray(Y, dtype=np.float64)
    out = np.zeros(wr.shape[0])
    lib.hsrq_oracle_residual(n, _ptr(H), n, wr.shape[0], _ptr(wr), _ptr(wi), _ptr(Y), n, _ptr(out))
    return out


def hnorm_inf(H):
    lib = _load()
    H = _fortran(H)
    return float(lib.hsrq_oracle_hnorm_inf(H.shape[0], _ptr(H), H.shape[0]))


def hsrq3in(H, wr, wi, S, ntries=None):
    """Inverse iteration with restarts (Sec. 4.2, Algorithm 14).

    Every shift is solved from the starting vector S[:, 0]; the shifts whose
    result fails the convergence test are solved again from S[:, 1], those
    that fail again from S[:, 2], up to S[:, ntries - 1].  A complex shift
    starts from the real vector (imaginary part zero), as in Sec. 4.3.
    Returns (Y, E, mu, info, tries) in the caller's column layout; tries[l] is
    the 0-based try whose result is returned (the last one tried when none
    converged, with info NOT_CONVERGED).
    """
    H = _fortran(H)
    n = H.shape[0]
    wr = np.asarray(wr, dtype=np.float64)
    wi = np.asarray(wi, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    m = wr.shape[0]
    ntries = S.shape[1] if ntries is None else ntries
    cols, ncols = columns_of(wi)
    Y = np.zeros((n, ncols))
    E = np.zeros(m, dtype=np.int32)
    mu = np.zeros(m)
    info = np.zeros(m, dtype=np.int32)
    tries = np.zeros(m, dtype=np.int32)
    act = list(range(m))
    for t in range(ntries):
        if not act:
            break
        wr_a, wi_a = wr[act], wi[act]
        ca, nca = columns_of(wi_a)
        B = np.zeros((n, nca))
        for k in range(len(act)):
            B[:, ca[k]] = S[:, t]
        Ya, Ea, mua, infoa = batch(H, wr_a, wi_a, B)
        for k, l in enumerate(act):
            w = 2 if wi[l] != 0.0 else 1
            Y[:, cols[l]:cols[l] + w] = Ya[:, ca[k]:ca[k] + w]
            E[l], mu[l], info[l], tries[l] = Ea[k], mua[k], infoa[k], t
        act = [l for k, l in enumerate(act) if infoa[k] == NOT_CONVERGED]
    return Y, E, mu, info, tries


def hessenberg_reduce(A):
    """Householder reduction to upper Hessenberg form, H = Q0^T A Q0 (the
    step before the solve, Sec. 1), one column at a time in plain numpy.

    For k = 0 .. n-3 the reflector H_k = I - tau_k u u^T, u = [1; v], maps
    x = A(k+1:n, k) to beta e_1 with beta = -sign(x_1) ||x|| (so x_1 - beta
    does not cancel): tau_k = (beta - x_1) / beta, v = x(2:) / (x_1 - beta).
    It is applied from the right to A(:, k+1:n), then from the left to
    A(k+1:n, k+1:n).  Returns (R, tau) in LAPACK's DGEHRD layout: H on and
    above the first subdiagonal of R, v below it in column k; tau has n - 1
    entries, the last 0.
    """
    R = np.array(A, dtype=np.float64, order="F", copy=True)
    n = R.shape[0]
    tau = np.zeros(max(n - 1, 1))
    for k in range(n - 2):
        x = R[k + 1:, k].copy()
        alpha = x[0]
        xnorm = np.linalg.norm(x[1:])
        if xnorm == 0.0:
            continue
        beta = -np.copysign(np.hypot(alpha, xnorm), alpha)
        t = (beta - alpha) / beta
        v = x[1:] / (alpha - beta)
        u = np.concatenate([[1.0], v])
        # from the right, then from the left
        R[:, k + 1:] -= t * np.outer(R[:, k + 1:] @ u, u)
        R[k + 1:, k + 1:] -= t * np.outer(u, u @ R[k + 1:, k + 1:])
        R[k + 1, k] = beta
        R[k + 2:, k] = v
        tau[k] = t
    return R, tau


def hessenberg_part(R):
    """H from the layout of hessenberg_reduce (zeros below the subdiagonal)."""
    return np.triu(R, -1)


def apply_q(R, tau, Z):
    """Q0 Z = H_0 (H_1 ( ... (H_{n-3} Z))) from the reflectors of
    hessenberg_reduce (the back-transform z = Q0 x of Sec. 1)."""
    Z = np.array(Z, dtype=np.float64, copy=True)
    n = R.shape[0]
    for k in range(n - 3, -1, -1):
        u = np.concatenate([[1.0], R[k + 2:, k]])
        Z[k + 1:] -= tau[k] * np.outer(u, u @ Z[k + 1:])
    return Z
