/*
 * hsrq_oracle.c -- plain, slow, untiled FP64 reference for the shifted
 * Hessenberg solves of "Robust level-3 BLAS inverse iteration from the
 * Hessenberg matrix" (Schwarz, arXiv 2101.05063).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or helper with the
 * GPU library.
 *
 * What it computes, per shift lambda (real, or complex with one member of a
 * conjugate pair) and starting vector b:
 *   the solution x of (H - lambda I) x = b by Henry's RQ approach (Sec. 2.2,
 *   Algorithm 1): Givens rotations applied from the right, column by column
 *   from n down to 2, each finished column of R used at once in a column
 *   oriented back substitution; then x(1) / R(1,1); then the back-transform
 *   x <- G_n^T ( ... (G_2^T y)).
 *   Overflow protection (Sec. 4.1): the iterate carries an integer exponent e
 *   with x_true = 2^e * x; before every division and every linear update the
 *   possible growth is bounded and the whole vector is rescaled by an exact
 *   power of two when the bound could reach 2^BIGEXP.
 *   Output (Sec. 4.1-4.2, Algorithm 11): the unit 2-norm vector
 *   y = x_true / ||x_true||_2 and ||x_true||_2 = mu * 2^E with mu in [0.5,1).
 *   Complex shifts (Sec. 4.3): rotations [[c, -s],[s, conj(c)]] with c complex
 *   and s real (the convention of eq. cgivens); everything else in complex
 *   arithmetic.
 *
 * Readings of the paper taken here (where it is silent or ambiguous):
 *   - Givens convention: r = hypot(a, |v|) >= 0, c = v / r, s = -a / r, so
 *     [a v] G = [0 r] and every R(k,k), k >= 2, is r > 0.  The hypot is
 *     written out: scale by 2^-ilogb(max), sqrt(fma(a,a, fma(vr,vr, vi*vi))),
 *     divide, unscale.  No libm hypot.
 *   - The rotated working column is updated as v(i) <- fma(s, v(i), c*h(i)),
 *     complex: per part, and on the shifted diagonal entry the complex
 *     product c*(h - lambda) is t_re = fma(c_re, hr, c_im*li),
 *     t_im = fma(c_im, hr, -(c_re*li)).  These are the exact scalar forms the
 *     rotations, the diagonal R(k,k) and the working column are defined by,
 *     so recorded values can be compared bit for bit.
 *   - Back substitution multipliers tau1 = s x(k), tau2 = conj(c) x(k) (the
 *     finished column of R is -s h(:,k-1) + conj(c) v).
 *   - The last back-transformed entry is stored (y(n) <- tau1), which the
 *     printed algorithms omit.
 *   - R(1,1) == 0 exactly: the shift is an exact eigenvalue of the computed
 *     factorisation; the result is the null vector Q^H e_1, info = 2.
 *   - Convergence (Sec. 4.2): ||x_true||_2 / ||b||_2 >= 1 / (10 n eps ||H||_inf)
 *     with eps = 2^-52; this is the paper's test rewritten without the
 *     assumption that b = ||H||_inf eps e.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC -pthread
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>
#include <limits.h>

#define BIGEXP 1000          /* keep every stored |component| below 2^BIGEXP */
#define NEG_EXP (-100000)    /* "exponent" of zero */

enum { OK = 0, NOT_CONVERGED = 1, SINGULAR = 2, NONFINITE = 3, REDUCED = 4 };

/* Upper exponent: |x| < 2^ub(x) for x != 0 (ilogb(x) + 1). */
static int ub(double x) {
    x = fabs(x);
    if (x == 0.0) return NEG_EXP;
    return ilogb(x) + 1;
}

static double maxd(double a, double b) { return a > b ? a : b; }

/*
 * Givens rotation for a real subdiagonal a != 0 and a complex (vr, vi):
 * [a v] [[c, -s],[s, conj(c)]] = [0 r]  (real case: vi = 0, c_im = 0).
 */
static void givens(double a, double vr, double vi,
                   double* c_re, double* c_im, double* s, double* r) {
    double m = maxd(fabs(a), maxd(fabs(vr), fabs(vi)));
    int e = ilogb(m);
    double as = ldexp(a, -e), vrs = ldexp(vr, -e), vis = ldexp(vi, -e);
    double q = vis * vis;
    q = fma(vrs, vrs, q);
    q = fma(as, as, q);
    double rs = sqrt(q);
    *c_re = vrs / rs;
    *c_im = vis / rs;
    *s = -as / rs;
    *r = ldexp(rs, e);
}

/* Complex helpers (plain arithmetic, no fused forms needed: x is compared to
   tolerance, not bitwise). */
static void cmul(double ar, double ai, double br, double bi, double* cr, double* ci) {
    double r = ar * br - ai * bi;
    double i = ar * bi + ai * br;
    *cr = r; *ci = i;
}

/* Smith's complex division (a / b). */
static void cdiv(double ar, double ai, double br, double bi, double* cr, double* ci) {
    if (fabs(br) >= fabs(bi)) {
        double t = bi / br, d = br + bi * t;
        *cr = (ar + ai * t) / d;
        *ci = (ai - ar * t) / d;
    } else {
        double t = br / bi, d = bi + br * t;
        *cr = (ar * t + ai) / d;
        *ci = (ai * t - ar) / d;
    }
}

static void scale_vec(int n, double* xr, double* xi, int p) {
    for (int i = 0; i < n; ++i) {
        xr[i] = ldexp(xr[i], -p);
        if (xi) xi[i] = ldexp(xi[i], -p);
    }
}

/* ||x||_2 of a (possibly complex) vector, scaled sum of squares. */
static double nrm2(int n, const double* xr, const double* xi) {
    double xmax = 0.0;
    for (int i = 0; i < n; ++i) {
        xmax = maxd(xmax, fabs(xr[i]));
        if (xi) xmax = maxd(xmax, fabs(xi[i]));
    }
    if (xmax == 0.0 || !isfinite(xmax)) return xmax;
    double ssq = 0.0;
    for (int i = 0; i < n; ++i) {
        double t = xr[i] / xmax;
        ssq += t * t;
        if (xi) { t = xi[i] / xmax; ssq += t * t; }
    }
    return xmax * sqrt(ssq);
}

/* ||H||_inf over the Hessenberg part (max row sum of |h(i,j)|, j >= i-1). */
double hsrq_oracle_hnorm_inf(int n, const double* H, int ldh) {
    double best = 0.0;
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = (i > 0 ? i - 1 : 0); j < n; ++j) s += fabs(H[i + (size_t)j * ldh]);
        best = maxd(best, s);
    }
    return best;
}

/* Returns OK, NONFINITE or REDUCED for the Hessenberg part of H. */
int hsrq_oracle_check(int n, const double* H, int ldh) {
    for (int j = 0; j < n; ++j)
        for (int i = 0; i <= j + 1 && i < n; ++i)
            if (!isfinite(H[i + (size_t)j * ldh])) return NONFINITE;
    for (int k = 1; k < n; ++k)
        if (H[k + (size_t)(k - 1) * ldh] == 0.0) return REDUCED;
    return OK;
}

/*
 * One shift.  b_im / y_im / v_im may be NULL for a real shift with a real
 * right-hand side (then li must be 0).  Record arrays are optional (NULL):
 *   rec_cre, rec_cim, rec_s, rec_phi : length n, index k = 0..n-1 (0-based
 *       column index of the rotation G_k acting on columns k-1 and k;
 *       entry 0 is padding c = 1, s = 0, phi = R(1,1) real part).
 *   snap_* : nsnap boundaries; snap_k[t] = b (0 < b <= n): the working column
 *       v(0:b-1) at the moment all rotations with index >= b have been
 *       applied is copied to snap_re/snap_im at offset snap_off[t].
 */
static int solve_one(int n, const double* H, int ldh, double lr, double li,
                     const double* b_re, const double* b_im,
                     double* y_re, double* y_im,
                     double hnorm, int32_t* E_out, double* mu_out,
                     double* rec_cre, double* rec_cim, double* rec_s, double* rec_phi,
                     int nsnap, const int* snap_k, const long* snap_off,
                     double* snap_re, double* snap_im,
                     double* work) {
    const int cplx = (li != 0.0) || (b_im != NULL);
    double* vr = work;
    double* vi = work + n;
    double* xr = work + 2 * (size_t)n;
    double* xi = work + 3 * (size_t)n;
    double* Cr = work + 4 * (size_t)n;
    double* Ci = work + 5 * (size_t)n;
    double* S = work + 6 * (size_t)n;
    long e = 0;
    int info = OK;
#define HH(i, j) H[(i) + (size_t)(j) * ldh]

    for (int i = 0; i < n; ++i) {
        vr[i] = HH(i, n - 1);
        vi[i] = 0.0;
        xr[i] = b_re[i];
        xi[i] = b_im ? b_im[i] : 0.0;
    }
    vr[n - 1] = HH(n - 1, n - 1) - lr;
    vi[n - 1] = -li;
    Cr[0] = 1.0; Ci[0] = 0.0; S[0] = 0.0;

    int snap_next = 0;
    /* snapshots are requested in decreasing boundary order */
    for (int k = n - 1; k >= 0; --k) {
        while (snap_next < nsnap && snap_k[snap_next] == k + 1) {
            int bnd = snap_k[snap_next];
            for (int i = 0; i < bnd; ++i) {
                snap_re[snap_off[snap_next] + i] = vr[i];
                if (snap_im) snap_im[snap_off[snap_next] + i] = vi[i];
            }
            ++snap_next;
        }
        if (k == 0) break;
        /* -- rotation G_k: annihilate h(k,k-1) against v(k) -- */
        double a = HH(k, k - 1);
        double cr, ci, s, phi;
        givens(a, vr[k], vi[k], &cr, &ci, &s, &phi);
        Cr[k] = cr; Ci[k] = ci; S[k] = s;
        if (rec_phi) rec_phi[k] = phi;

        /* -- x(k) <- x(k) / R(k,k), guarded -- */
        double mag = maxd(fabs(xr[k]), fabs(xi[k]));
        if (mag != 0.0) {
            int p = ub(mag) - ilogb(phi) + 1 - BIGEXP;
            if (p > 0) { scale_vec(n, xr, cplx ? xi : NULL, p); e += p; }
        }
        xr[k] = xr[k] / phi;
        xi[k] = xi[k] / phi;

        /* -- multipliers of the finished column R(:,k) = -s h(:,k-1) + conj(c) v -- */
        double t1r = s * xr[k], t1i = s * xi[k];
        double t2r, t2i;
        cmul(cr, -ci, xr[k], xi[k], &t2r, &t2i);

        /* -- guard the update x(0:k-1) -= tau2 v - tau1 h~(:,k-1) -- */
        double xm = 0.0, vm = 0.0, hm = 0.0;
        for (int i = 0; i < k; ++i) {
            xm = maxd(xm, maxd(fabs(xr[i]), fabs(xi[i])));
            vm = maxd(vm, maxd(fabs(vr[i]), fabs(vi[i])));
            double h = (i == k - 1) ? fabs(HH(i, k - 1) - lr) + fabs(li) : fabs(HH(i, k - 1));
            hm = maxd(hm, h);
        }
        double t1m = maxd(fabs(t1r), fabs(t1i)), t2m = maxd(fabs(t2r), fabs(t2i));
        int eb = ub(xm);
        int e2 = (t2m != 0.0 && vm != 0.0) ? ub(t2m) + ub(vm) + 1 : NEG_EXP;
        int e3 = (t1m != 0.0 && hm != 0.0) ? ub(t1m) + ub(hm) + 1 : NEG_EXP;
        if (e2 > eb) eb = e2;
        if (e3 > eb) eb = e3;
        eb += 2;
        if (eb > BIGEXP) {
            int p = eb - BIGEXP;
            scale_vec(n, xr, cplx ? xi : NULL, p);
            t1r = ldexp(t1r, -p); t1i = ldexp(t1i, -p);
            t2r = ldexp(t2r, -p); t2i = ldexp(t2i, -p);
            e += p;
        }
        for (int i = 0; i < k; ++i) {
            double hr = HH(i, k - 1), hi = 0.0;
            if (i == k - 1) { hr = hr - lr; hi = -li; }
            double pr, pi, qr, qi;
            cmul(t2r, t2i, vr[i], vi[i], &pr, &pi);
            cmul(t1r, t1i, hr, hi, &qr, &qi);
            xr[i] = xr[i] - pr + qr;
            xi[i] = xi[i] - pi + qi;
        }
        /* -- rotate the working column into column k-1 -- */
        for (int i = 0; i < k - 1; ++i) {
            double h = HH(i, k - 1);
            vr[i] = fma(s, vr[i], cr * h);
            vi[i] = fma(s, vi[i], ci * h);
        }
        {
            double hr = HH(k - 1, k - 1) - lr;
            double tr = fma(cr, hr, ci * li);
            double ti = fma(ci, hr, -(cr * li));
            vr[k - 1] = fma(s, vr[k - 1], tr);
            vi[k - 1] = fma(s, vi[k - 1], ti);
        }
    }

    /* -- last pivot R(1,1) = v(1) -- */
    if (rec_phi) rec_phi[0] = vr[0];
    if (vr[0] == 0.0 && vi[0] == 0.0) {
        info = SINGULAR;
        for (int i = 0; i < n; ++i) { xr[i] = 0.0; xi[i] = 0.0; }
        xr[0] = 1.0;
    } else {
        double mag = maxd(fabs(xr[0]), fabs(xi[0]));
        if (mag != 0.0) {
            int lo = ilogb(maxd(fabs(vr[0]), fabs(vi[0])));
            int p = ub(mag) - lo + 2 - BIGEXP;
            if (p > 0) { scale_vec(n, xr, cplx ? xi : NULL, p); e += p; }
        }
        if (cplx) {
            double qr, qi;
            cdiv(xr[0], xi[0], vr[0], vi[0], &qr, &qi);
            xr[0] = qr; xi[0] = qi;
        } else {
            xr[0] = xr[0] / vr[0];
        }
    }

    /* -- normalise, then back-transform (rotations keep the 2-norm) -- */
    double nu = nrm2(n, xr, cplx ? xi : NULL);
    int32_t E;
    double mu;
    if (info == SINGULAR) {
        E = INT32_MAX; mu = 0.0; nu = 1.0;
    } else if (nu == 0.0) {
        E = 0; mu = 0.0; nu = 1.0; info = NOT_CONVERGED;
    } else {
        int lg = ilogb(nu);
        long EE = e + lg + 1;
        E = (EE > INT32_MAX - 1) ? INT32_MAX - 1 : (int32_t)EE;
        mu = ldexp(nu, -(lg + 1));
    }
    for (int i = 0; i < n; ++i) { xr[i] = xr[i] / nu; xi[i] = xi[i] / nu; }
    double t1r = xr[0], t1i = xi[0];
    for (int k = 1; k < n; ++k) {
        double t2r = xr[k], t2i = xi[k];
        double c_r = Cr[k], c_i = Ci[k], s = S[k];
        /* y(k-1) = c tau1 - s tau2 ; tau1 = s tau1 + conj(c) tau2 */
        double ar, ai, br, bi;
        cmul(c_r, c_i, t1r, t1i, &ar, &ai);
        xr[k - 1] = ar - s * t2r;
        xi[k - 1] = ai - s * t2i;
        cmul(c_r, -c_i, t2r, t2i, &br, &bi);
        t1r = s * t1r + br;
        t1i = s * t1i + bi;
    }
    xr[n - 1] = t1r; xi[n - 1] = t1i;
    for (int i = 0; i < n; ++i) {
        y_re[i] = xr[i];
        if (y_im) y_im[i] = xi[i];
    }
    if (rec_cre) for (int k = 0; k < n; ++k) { rec_cre[k] = Cr[k]; rec_s[k] = S[k]; }
    if (rec_cim) for (int k = 0; k < n; ++k) rec_cim[k] = Ci[k];

    /* -- convergence test (Varah's criterion in the paper's form) -- */
    if (info == OK) {
        double bn = nrm2(n, b_re, b_im);
        if (bn == 0.0 || hnorm == 0.0) {
            info = NOT_CONVERGED;
        } else {
            double lhs = (double)E + log2(mu) - log2(bn) + log2(10.0 * n) - 52.0 + log2(hnorm);
            if (!(lhs >= 0.0)) info = NOT_CONVERGED;
        }
    }
    *E_out = E;
    *mu_out = mu;
    return info;
#undef HH
}

/*
 * Single-shift entry point, exposed for the tests.
 */
int hsrq_oracle_solve1(int n, const double* H, int ldh, double lr, double li,
                       const double* b_re, const double* b_im,
                       double* y_re, double* y_im, int32_t* E, double* mu,
                       double* rec_cre, double* rec_cim, double* rec_s, double* rec_phi,
                       int nsnap, const int* snap_k, const long* snap_off,
                       double* snap_re, double* snap_im) {
    int st = hsrq_oracle_check(n, H, ldh);
    if (st != OK || !isfinite(lr) || !isfinite(li)) {
        for (int i = 0; i < n; ++i) { y_re[i] = 0.0; if (y_im) y_im[i] = 0.0; }
        *E = 0; *mu = 0.0;
        return st != OK ? st : NONFINITE;
    }
    double hn = hsrq_oracle_hnorm_inf(n, H, ldh);
    double* work = (double*)malloc(sizeof(double) * 7 * (size_t)(n > 0 ? n : 1));
    if (!work) return -1;
    int info = solve_one(n, H, ldh, lr, li, b_re, b_im, y_re, y_im, hn, E, mu,
                         rec_cre, rec_cim, rec_s, rec_phi, nsnap, snap_k, snap_off,
                         snap_re, snap_im, work);
    free(work);
    return info;
}

/* ---------------- many shifts, threaded over shifts ---------------- */

typedef struct {
    int n; const double* H; int ldh; int m;
    const double* wr; const double* wi;
    const double* B; int ldb;      /* starting vectors, caller's column layout */
    double* Y; int ldy;            /* results, same layout */
    int32_t* E; double* mu; int32_t* info;
    const long* col_of;            /* first column of shift l */
    double hnorm;
    int next;                      /* shared counter */
    pthread_mutex_t lock;
} batch_t;

static void* batch_worker(void* arg) {
    batch_t* bt = (batch_t*)arg;
    double* work = (double*)malloc(sizeof(double) * 7 * (size_t)bt->n);
    for (;;) {
        pthread_mutex_lock(&bt->lock);
        int l = bt->next++;
        pthread_mutex_unlock(&bt->lock);
        if (l >= bt->m) break;
        long col = bt->col_of[l];
        const double* bre = bt->B + (size_t)col * bt->ldb;
        double* yre = bt->Y + (size_t)col * bt->ldy;
        double li = bt->wi[l];
        if (li != 0.0) {
            /* complex: caller stores [re im] in adjacent columns; a negative
               imaginary part is the conjugate of the stored member. */
            const double* bim = bre + bt->ldb;
            double* yim = yre + bt->ldy;
            bt->info[l] = solve_one(bt->n, bt->H, bt->ldh, bt->wr[l], li, bre, bim, yre, yim,
                                    bt->hnorm, &bt->E[l], &bt->mu[l],
                                    NULL, NULL, NULL, NULL, 0, NULL, NULL, NULL, NULL, work);
        } else {
            bt->info[l] = solve_one(bt->n, bt->H, bt->ldh, bt->wr[l], 0.0, bre, NULL, yre, NULL,
                                    bt->hnorm, &bt->E[l], &bt->mu[l],
                                    NULL, NULL, NULL, NULL, 0, NULL, NULL, NULL, NULL, work);
        }
    }
    free(work);
    return NULL;
}

/*
 * m shifts on one matrix.  B/Y: n x ncols column-major, one column per real
 * shift, two adjacent [re im] columns per complex shift, in shift order.
 * Returns 0, or the input status (NONFINITE / REDUCED) applied to all shifts.
 */
int hsrq_oracle_batch(int n, const double* H, int ldh, int m,
                      const double* wr, const double* wi,
                      const double* B, int ldb, double* Y, int ldy,
                      int32_t* E, double* mu, int32_t* info, int nthreads) {
    long* col_of = (long*)malloc(sizeof(long) * (size_t)(m > 0 ? m : 1));
    long col = 0;
    for (int l = 0; l < m; ++l) { col_of[l] = col; col += (wi[l] != 0.0) ? 2 : 1; }
    int st = hsrq_oracle_check(n, H, ldh);
    for (int l = 0; l < m && st == OK; ++l)
        if (!isfinite(wr[l]) || !isfinite(wi[l])) st = NONFINITE;
    if (st != OK) {
        for (int l = 0; l < m; ++l) {
            info[l] = st; E[l] = 0; mu[l] = 0.0;
            int w = (wi[l] != 0.0) ? 2 : 1;
            for (int c = 0; c < w; ++c)
                for (int i = 0; i < n; ++i) Y[i + (size_t)(col_of[l] + c) * ldy] = 0.0;
        }
        free(col_of);
        return st;
    }
    batch_t bt;
    bt.n = n; bt.H = H; bt.ldh = ldh; bt.m = m; bt.wr = wr; bt.wi = wi;
    bt.B = B; bt.ldb = ldb; bt.Y = Y; bt.ldy = ldy; bt.E = E; bt.mu = mu; bt.info = info;
    bt.col_of = col_of; bt.hnorm = hsrq_oracle_hnorm_inf(n, H, ldh); bt.next = 0;
    pthread_mutex_init(&bt.lock, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > m) nthreads = m > 0 ? m : 1;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, batch_worker, &bt);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&bt.lock);
    free(col_of);
    return 0;
}

/*
 * Normalised residuals ||H y - lambda y||_2 / (||H||_F ||y||_2) per shift,
 * accumulated in long double.  Same column layout as hsrq_oracle_batch.
 */
int hsrq_oracle_residual(int n, const double* H, int ldh, int m,
                         const double* wr, const double* wi,
                         const double* Y, int ldy, double* out) {
    long double hf = 0.0L;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i <= j + 1 && i < n; ++i) {
            long double h = H[i + (size_t)j * ldh];
            hf += h * h;
        }
    hf = sqrtl(hf);
    long col = 0;
    for (int l = 0; l < m; ++l) {
        int cx = wi[l] != 0.0;
        const double* yr = Y + (size_t)col * ldy;
        const double* yi = cx ? yr + ldy : NULL;
        long double num = 0.0L, den = 0.0L;
        for (int i = 0; i < n; ++i) {
            long double ar = 0.0L, ai = 0.0L;
            int j0 = i > 0 ? i - 1 : 0;
            for (int j = j0; j < n; ++j) {
                long double h = H[i + (size_t)j * ldh];
                ar += h * yr[j];
                if (cx) ai += h * yi[j];
            }
            long double lr = wr[l], li = wi[l];
            long double y_r = yr[i], y_i = cx ? yi[i] : 0.0L;
            ar -= lr * y_r - li * y_i;
            ai -= lr * y_i + li * y_r;
            num += ar * ar + ai * ai;
            den += y_r * y_r + y_i * y_i;
        }
        out[l] = (double)(sqrtl(num) / (hf * sqrtl(den)));
        col += cx ? 2 : 1;
    }
    return 0;
}
