"""Comparison helpers for the GPU-vs-reference parity tests.

Tolerances (the accuracy targets of the solver, restated):
  * normalised residual ||H y - lambda y|| / (||H||_F ||y||) <= 10 n eps64
    for eigenvalue shifts;
  * direction agreement |y^H y_ref| / (||y|| ||y_ref||) >= 1 - 1e-10 for
    shifts separated by >= 1e-3 ||H|| (and for shifts far from the spectrum);
  * scale exponent bit-exact; when the two differ the true norm must sit
    within rounding distance of a power of two (a "straddle"), which the
    helper reports instead of hiding;
  * rotations, the diagonal of R and the working columns bit-exact.
"""
import numpy as np

EPS = 2.0 ** -52


def direction(y, z):
    ny, nz = np.linalg.norm(y), np.linalg.norm(z)
    if ny == 0 or nz == 0:
        return 0.0
    return abs(np.vdot(y, z)) / (ny * nz)


def vec(Y, cols, wi, l):
    c = cols[l]
    return Y[:, c] + 1j * Y[:, c + 1] if wi[l] != 0 else Y[:, c]


# a scale exponent may differ from the reference's by one only when log2 of the
# true norm lies within this distance of an integer (the FP64 paths: the two
# norms differ by GEMM summation order, ~1e-13 relative, so 1e-6 in log2
# leaves a wide margin while still catching any real mismatch)
STRADDLE_TOL = 1e-6


def compare(Yg, Eg, mug, infog, Yo, Eo, muo, infoo, wi, dir_tol=1e-10, sel=None, mu_tol=1e-12,
            straddle_tol=STRADDLE_TOL):
    """Compare per shift; returns dict(straddles=[...]) and raises on failure."""
    from oracle.oracle import columns_of
    cols, _ = columns_of(wi)
    m = len(wi)
    straddles = []
    idx = range(m) if sel is None else sel
    for l in idx:
        assert infog[l] == infoo[l], (l, infog[l], infoo[l])
        if infoo[l] in (3, 4):
            continue
        if infoo[l] == 2:
            assert Eg[l] == Eo[l]
        elif Eg[l] != Eo[l]:
            # a straddle: |log2 ||x|| - integer| tiny
            lg = Eo[l] + np.log2(muo[l])
            assert abs(Eg[l] - Eo[l]) == 1 and abs(lg - round(lg)) < straddle_tol, (l, Eg[l], Eo[l], muo[l], mug[l])
            straddles.append(l)
        else:
            assert abs(mug[l] - muo[l]) <= mu_tol * muo[l] + 1e-300, (l, mug[l], muo[l])
        d = direction(vec(Yg, cols, wi, l), vec(Yo, cols, wi, l))
        assert d >= 1.0 - dir_tol, (l, 1.0 - d)
    return dict(straddles=straddles)
