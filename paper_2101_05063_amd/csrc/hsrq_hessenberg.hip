// hsrq_hessenberg.hip -- the steps around the solve (Sec. 1): the reduction
// of a general real matrix to upper Hessenberg form, H = Q0^T A Q0, and the
// back-transform z = Q0 x of eigenvectors of H into eigenvectors of A.
//
// Q0 = H_0 H_1 ... H_{n-3}, H_k = I - tau_k u_k u_k^T with u_k zero above
// row k+1, u_k(k+1) = 1 and u_k(k+2:n) stored below the subdiagonal of
// column k of the reduced matrix (the storage of LAPACK's DGEHRD).  H_k is
// chosen so that H_k A(k+1:n, k) = beta e_1 with beta = -sign(alpha) ||x||,
// alpha = A(k+1, k) (no cancellation in alpha - beta).
//
// Applying H_k from both sides is one rank-2 update of the trailing columns:
// with y = A(:, k+1:n) u and z = u^T A(k+1:n, k+1:n) (both from A before the
// step) and s = u^T y(k+1:n),
//   A(:, k+1:n)      -= tau y u^T                     (from the right)
//   A(k+1:n, k+1:n)  -= tau u w^T,  w = z - tau s u   (then from the left).
// The reduction is HBM-bound, so every column costs one read and one write of
// the trailing matrix: the sweep that applies step k to columns k+2..n-1 also
// forms the partial sums of y and z for step k+1 (whose reflector is known
// once column k+1 alone has been updated).  Per column:
//   k_reduce      y, z of step k from the partial sums (fixed order)
//   k_colhouse_r  s; column k+1 updated; the reflector of column k+1 (the
//                 column in registers; k_colhouse above 8192 rows)
//   k_sweep       columns k+2..n-1 updated; partial sums for step k+1
//                 (non-temporal accesses while the trailing part is large)
// Every reduction has a fixed order, so the results are the same on every
// run.  The back-transform is blocked (compact WY): panels of 128
// reflectors; k_vpanel makes a panel explicit, k_larft builds the
// triangular factor T of every panel in one launch, and the products with
// the vectors run on rocBLAS DGEMM (k_sumsplit adds the row-chunk partials
// of the short, wide products).
#include <hip/hip_runtime.h>
#include <math.h>

#include <rocblas/rocblas.h>

#include "hsrq.h"
#include "hsrq_plan.h"

namespace hsrq {
namespace {

constexpr int kT = 64;     // sweep tiles: 64 rows x 64 columns, 256 threads
constexpr double kNTBytes = 256.0 * 1024 * 1024;  // sweeps past this size use non-temporal hints
constexpr int kCH = 1024;  // threads of k_colhouse

__device__ __forceinline__ double wsum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ double wmax(double x) {
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}
// block sum / max over kCH threads in a fixed order (every thread gets it)
__device__ __forceinline__ double block_sum(double x, double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  x = wsum(x);
  __syncthreads();
  if (lane == 0) red[w] = x;
  __syncthreads();
  double t = 0.0;
  for (int j = 0; j < kCH / 64; ++j) t += red[j];
  return t;
}
__device__ __forceinline__ double block_max(double x, double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  x = wmax(x);
  __syncthreads();
  if (lane == 0) red[w] = x;
  __syncthreads();
  double t = 0.0;
  for (int j = 0; j < kCH / 64; ++j) t = fmax(t, red[j]);
  return t;
}

// One element of the rank-2 update of step k: tyr = tau y(r), tur = tau
// u(r) (0 above row k+1), uc = u(c), wc = w(c).
__device__ __forceinline__ double rank2(double a, double tyr, double uc, double tur, double wc) {
  a = fma(-tyr, uc, a);
  return fma(-tur, wc, a);
}

// Step q's s = u^T y(q+1:n), column q+1 updated with step q, and the
// reflector of column q+1 (when q+1 <= n-3).  q = -1: only the reflector of
// column 0.  One block of kCH threads; thread t owns rows t, t + kCH, ...
// in both phases, so it reads back only what it wrote itself.
__global__ void __launch_bounds__(kCH) k_colhouse(double* A, long long lda, int n, int q, double* tau,
                                                  const double* uq, double* un, const double* y,
                                                  const double* z, double* sc) {
  __shared__ double red[kCH / 64];
  __shared__ double alpha_s;
  const int tid = threadIdx.x;
  const int c = q + 1;  // the column updated here and reduced next
  double* col = A + (long long)c * lda;
  if (q >= 0) {
    const int m = n - q - 1;
    double sp = 0.0;
    for (int i = tid; i < m; i += kCH) sp = fma(uq[i], y[q + 1 + i], sp);
    const double s = block_sum(sp, red);
    const double t = tau[q];
    if (tid == 0) sc[0] = s;
    const double w0 = fma(-(t * s), uq[0], z[0]);
    for (int r = tid; r < n; r += kCH) {
      const double tur = r >= q + 1 ? t * uq[r - (q + 1)] : 0.0;
      col[r] = rank2(col[r], t * y[r], uq[0], tur, w0);
    }
  }
  if (c > n - 3) return;  // no reflector for this column
  // the reflector of column c: x = A(c+1:n, c), m entries
  const int m = n - c - 1;
  double* x = col + (c + 1);
  if (tid == ((c + 1) % kCH)) alpha_s = col[c + 1];  // the thread that owns row c+1
  double mx = 0.0;
  for (int r = tid; r < n; r += kCH)
    if (r >= c + 2) mx = fmax(mx, fabs(col[r]));
  mx = block_max(mx, red);
  double ss = 0.0;
  if (mx > 0.0)
    for (int r = tid; r < n; r += kCH)
      if (r >= c + 2) {
        const double v = col[r] / mx;
        ss = fma(v, v, ss);
      }
  ss = block_sum(ss, red);  // its first barrier also publishes alpha_s
  const double xnorm = mx * sqrt(ss);
  const double alpha = alpha_s;
  double t = 0.0, beta = alpha, scal = 0.0;
  if (xnorm != 0.0) {
    // |beta| = hypot(alpha, xnorm), written out with a power-of-two scale
    const double big = fmax(fabs(alpha), xnorm);
    const int e = ilogb(big);
    const double as = ldexp(alpha, -e), xs = ldexp(xnorm, -e);
    const double r = ldexp(sqrt(fma(as, as, xs * xs)), e);
    beta = alpha >= 0.0 ? -r : r;
    t = (beta - alpha) / beta;
    scal = 1.0 / (alpha - beta);
  }
  for (int r = tid; r < n; r += kCH)
    if (r >= c + 2) {
      const double v = col[r] * scal;
      col[r] = v;
      un[r - (c + 1)] = v;
    }
  if (tid == 0) {
    tau[c] = t;
    x[0] = beta;
    un[0] = 1.0;
  }
  (void)m;
}

// Column sums over the 64 rows of a tile for the CW = 16 columns of a wave,
// through lane exchanges alone (no shared memory): four halving steps over
// lane bits 5, 4, 3, 2 leave lane l with the sum of column l >> 2 over the
// 16 lanes that agree with it in those bits... (each step keeps the half of
// the columns its bit selects and adds the partner's copy of that half),
// then the 4 lanes of a column are added.  A fixed order, so the result
// does not depend on the schedule.  Returns the sum of column (lane >> 2)
// in every lane (the caller stores it from the lanes with (lane & 3) == 0).
constexpr int kCW = 16;  // columns per wave in the sweeps
__device__ __forceinline__ double tile_colsum(const double* v) {
  const int l = threadIdx.x & 63;
  double w8[8], w4[4], w2[2];
  const bool b5 = (l & 32) != 0, b4 = (l & 16) != 0, b3 = (l & 8) != 0, b2 = (l & 4) != 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) w8[j] = (b5 ? v[j + 8] : v[j]) + __shfl_xor(b5 ? v[j] : v[j + 8], 32, 64);
#pragma unroll
  for (int j = 0; j < 4; ++j) w4[j] = (b4 ? w8[j + 4] : w8[j]) + __shfl_xor(b4 ? w8[j] : w8[j + 4], 16, 64);
#pragma unroll
  for (int j = 0; j < 2; ++j) w2[j] = (b3 ? w4[j + 2] : w4[j]) + __shfl_xor(b3 ? w4[j] : w4[j + 2], 8, 64);
  double s = (b2 ? w2[1] : w2[0]) + __shfl_xor(b2 ? w2[0] : w2[1], 4, 64);
  s += __shfl_xor(s, 1, 64);
  s += __shfl_xor(s, 2, 64);
  return s;
}

// k_colhouse for n <= R kCH: the column lives in registers (thread t owns
// rows t + j kCH, j < R), so it is read once and written once.  The same
// steps as k_colhouse, with the norm of x taken in one pass (sum of squares
// and largest magnitude reduced together) and redone with a power-of-two
// scale only when the largest magnitude lies outside [2^-480, 2^480], where
// a square could overflow or lose to underflow; row c+1 (alpha, then beta)
// is written by the thread that owns it.
template <int R>
__global__ void __launch_bounds__(kCH) k_colhouse_r(double* A, long long lda, int n, int q, double* tau,
                                                    const double* uq, double* un, const double* y,
                                                    const double* z, double* sc) {
  __shared__ double red0[kCH / 64], red1[kCH / 64], red2[kCH / 64], red3[kCH / 64];
  __shared__ double alpha_s;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c = q + 1;  // the column updated here and reduced next
  const bool refl = c <= n - 3;
  double* col = A + (long long)c * lda;
  double a[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int r = tid + j * kCH;
    a[j] = r < n ? col[r] : 0.0;
  }
  if (q >= 0) {
    // y and u of the thread's rows stay in registers beside the column (84
    // registers per lane at R = 8, of the 128 a 1024-thread block allows)
    double yv[R], uv[R], sp = 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int r = tid + j * kCH;
      const double yr = r < n ? y[r] : 0.0;
      const double ur = (r < n && r >= q + 1) ? uq[r - (q + 1)] : 0.0;
      yv[j] = yr;
      uv[j] = ur;
      sp = fma(ur, yr, sp);
    }
    sp = wsum(sp);
    if (lane == 0) red0[w] = sp;
    __syncthreads();
    double s = 0.0;
    for (int j = 0; j < kCH / 64; ++j) s += red0[j];
    const double t = tau[q];
    if (tid == 0) sc[0] = s;
    const double u0 = uq[0];
    const double w0 = fma(-(t * s), u0, z[0]);
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int r = tid + j * kCH;
      a[j] = rank2(a[j], t * yv[j], u0, t * uv[j], w0);
      if (r < n && (!refl || r <= c)) col[r] = a[j];
    }
  }
  if (!refl) return;  // no reflector for this column
  double ss = 0.0, mx = 0.0;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int r = tid + j * kCH;
    if (r == c + 1) alpha_s = a[j];
    if (r >= c + 2 && r < n) {
      ss = fma(a[j], a[j], ss);
      mx = fmax(mx, fabs(a[j]));
    }
  }
  ss = wsum(ss);
  mx = wmax(mx);
  if (lane == 0) {
    red1[w] = ss;
    red2[w] = mx;
  }
  __syncthreads();  // also publishes alpha_s
  ss = 0.0;
  mx = 0.0;
  for (int j = 0; j < kCH / 64; ++j) {
    ss += red1[j];
    mx = fmax(mx, red2[j]);
  }
  double xnorm = 0.0;
  if (mx > 0.0) {
    if (mx >= 0x1p-480 && mx <= 0x1p480) {
      xnorm = sqrt(ss);
    } else {  // scaled by 2^-e, exact
      const int e = ilogb(mx);
      double s2 = 0.0;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const int r = tid + j * kCH;
        if (r >= c + 2 && r < n) {
          const double v = ldexp(a[j], -e);
          s2 = fma(v, v, s2);
        }
      }
      s2 = wsum(s2);
      if (lane == 0) red3[w] = s2;
      __syncthreads();
      s2 = 0.0;
      for (int j = 0; j < kCH / 64; ++j) s2 += red3[j];
      xnorm = ldexp(sqrt(s2), e);
    }
  }
  const double alpha = alpha_s;
  double t = 0.0, beta = alpha, scal = 0.0;
  if (xnorm != 0.0) {
    // |beta| = hypot(alpha, xnorm), written out with a power-of-two scale
    const double big = fmax(fabs(alpha), xnorm);
    const int e = ilogb(big);
    const double as = ldexp(alpha, -e), xs = ldexp(xnorm, -e);
    const double rr = ldexp(sqrt(fma(as, as, xs * xs)), e);
    beta = alpha >= 0.0 ? -rr : rr;
    t = (beta - alpha) / beta;
    scal = 1.0 / (alpha - beta);
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int r = tid + j * kCH;
    if (r == c + 1) col[r] = beta;
    if (r >= c + 2 && r < n) {
      const double v = a[j] * scal;
      col[r] = v;
      un[r - (c + 1)] = v;
    }
  }
  if (tid == 0) {
    tau[c] = t;
    un[0] = 1.0;
  }
}

// The sweep of step k over columns k+2..n-1 (all rows), 64 x 64 tiles: lane
// = row, wave w = 16 columns.  UPD: apply step k (tau[k], u0 = u_k, y, z, s).
// ACC: partial sums for step k+1 (u1 = u_{k+1}): py[ct][r] = sum over the
// tile's columns of A(r, c) u1(c), pz[rt][c'] = sum over the tile's rows of
// u1(r) A(r, c).  k = -1 with UPD false: the partial sums of step 0.  The
// per-column values are wave-uniform; the 16 loads of a lane are issued
// before any of them is used.
template <bool UPD, bool ACC, bool NT>
__global__ void __launch_bounds__(256) k_sweep(double* __restrict__ A, long long lda, int n, int k,
                                               const double* __restrict__ tau, const double* __restrict__ u0,
                                               const double* __restrict__ u1, const double* __restrict__ y,
                                               const double* __restrict__ z, const double* __restrict__ sc,
                                               double* __restrict__ py, double* __restrict__ pz) {
  __shared__ double red[4][kT];
  const int l = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = blockIdx.x * kT + l;
  const int c0 = k + 2;
  const int cb = c0 + blockIdx.y * kT + w * kCW;
  const bool rok = r < n;
  const int rr = rok ? r : n - 1;
  double tyr = 0.0, tur = 0.0, ts = 0.0, ur1 = 0.0;
  if (UPD) {
    const double t = tau[k];
    ts = t * sc[0];
    tyr = rok ? t * y[rr] : 0.0;
    tur = (rok && r >= k + 1) ? t * u0[rr - (k + 1)] : 0.0;
  }
  if (ACC) ur1 = (rok && r >= k + 2) ? u1[rr - (k + 2)] : 0.0;
  double a[kCW], uc[kCW], wc[kCW], vc[kCW];
#pragma unroll
  for (int j = 0; j < kCW; ++j) {
    const int c = cb + j < n ? cb + j : n - 1;  // clamped: columns past n are never stored
    a[j] = NT ? __builtin_nontemporal_load(&A[(long long)c * lda + rr]) : A[(long long)c * lda + rr];
    if (UPD) {
      uc[j] = u0[c - (k + 1)];
      wc[j] = fma(-ts, uc[j], z[c - (k + 1)]);
    }
    if (ACC) vc[j] = u1[c - (k + 2)];
  }
  double ys = 0.0, zp[kCW];
#pragma unroll
  for (int j = 0; j < kCW; ++j) {
    const int c = cb + j;
    const bool cok = c < n;  // uniform over the wave
    if (UPD) {
      a[j] = rank2(a[j], tyr, uc[j], tur, wc[j]);
      if (rok && cok) {
        if (NT)
          __builtin_nontemporal_store(a[j], &A[(long long)c * lda + r]);
        else
          A[(long long)c * lda + r] = a[j];
      }
    }
    const double uv = (rok && cok) ? a[j] : 0.0;
    if (ACC) {
      ys = fma(uv, vc[j], ys);
      zp[j] = ur1 * uv;
    }
  }
  if (ACC) {
    const double zs = tile_colsum(zp);
    const int c = cb + (l >> 2);
    if ((l & 3) == 0 && c < n) pz[(long long)blockIdx.x * n + (c - (k + 2))] = zs;
    red[w][l] = ys;
    __syncthreads();
    if (w == 0 && rok) py[(long long)blockIdx.y * n + r] = (red[0][l] + red[1][l]) + (red[2][l] + red[3][l]);
  }
}

// y(i) = sum_ct py[ct][i] (i < ny; rows of py ny apart), z(c) = sum_rt
// pz[rt][c] (c < m; rows of pz lz apart).  A block sums 32 outputs; its 8
// groups of 32 threads each sum every 8th partial (in order) and the 8 sums
// are added in a fixed order, so the result does not depend on the
// schedule.
constexpr int kRO = 32;  // outputs per reduction block
constexpr int kRG = 8;   // partial groups per output
__global__ void __launch_bounds__(kRO * kRG) k_reduce(const double* py, int nct, int ny, const double* pz, int nrt,
                                                      long long lz, int m, double* y, double* z) {
  __shared__ double part[kRG][kRO];
  const int o = threadIdx.x % kRO, g = threadIdx.x / kRO;
  const int i = blockIdx.x * kRO + o;
  double s = 0.0;
  if (i < ny) {
#pragma unroll 4
    for (int ct = g; ct < nct; ct += kRG) s += py[(long long)ct * ny + i];
  } else if (i < ny + m) {
    const int c = i - ny;
#pragma unroll 4
    for (int rt = g; rt < nrt; rt += kRG) s += pz[rt * lz + c];
  }
  part[g][o] = s;
  __syncthreads();
  if (g == 0 && i < ny + m) {
    const double t = ((part[0][o] + part[1][o]) + (part[2][o] + part[3][o])) +
                     ((part[4][o] + part[5][o]) + (part[6][o] + part[7][o]));
    if (i < ny)
      y[i] = t;
    else
      z[i - ny] = t;
  }
}

// The back-transform in compact WY form: reflectors j0 .. j0+kb-1 applied
// together are I - V T V^T (V = [u_j0 .. u_j0+kb-1], T upper triangular,
// LAPACK's DLARFT, forward and columnwise), so that Z <- (I - V T V^T) Z is
// three matrix products.  V is zero above row j0+1; the panel holds rows
// j0+1 .. n-1 only.
constexpr int kWY = 128;  // reflectors per panel (T's block: 132 KB of shared memory)

// V (column-major nr x kb, nr = n - j0 - 1): u_k explicit, 0 above its unit
// entry at row k+1, A(r, k) below it
__global__ void __launch_bounds__(256) k_vpanel(const double* __restrict__ A, long long lda, int n, int j0, int kb,
                                                double* __restrict__ V) {
  const long long nr = n - (j0 + 1);
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= nr * kb) return;
  const int c = (int)(e / nr);
  const int i = j0 + 1 + (int)(e - (long long)c * nr);  // the row of A
  const int k = j0 + c;                                  // the reflector
  V[e] = i == k + 1 ? 1.0 : (i > k + 1 ? A[i + (long long)k * lda] : 0.0);
}

// T (column-major kb x kb, zero below the diagonal) from G = V^T V and the
// panel's tau: T(i, i) = tau_i and, for i < j, T(i, j) = -tau_j times the
// sum over i <= k < j of T(i, k) G(k, j).  Row i of T needs only its own
// earlier entries, so the rows run side by side in one block, kLP threads
// per row; thread part p handles the columns k = p mod kLP, reads only the
// entries of its row that it wrote itself, and takes its columns four at
// a time (terms outside i <= k < j are zero), so that a step's
// shared-memory loads are in flight together.  The partial sums are
// combined in a fixed order.
constexpr int kLP = 4;          // threads per row of T
constexpr int kLM = kWY / kLP;  // columns per thread
// the panels: panel p holds reflectors j0 .. jhi, jhi = n - 3 - p kWY, j0 =
// max(0, jhi - kWY + 1); npanels(n) of them
__host__ __device__ inline int npanels(int n) { return n >= 3 ? (n - 2 + kWY - 1) / kWY : 0; }
__host__ __device__ inline void panel(int n, int p, int& j0, int& kb) {
  const int jhi = n - 3 - p * kWY;
  j0 = jhi - kWY + 1 > 0 ? jhi - kWY + 1 : 0;
  kb = jhi - j0 + 1;
}
// one block per panel: G and T of panel p at Gs + p kWY^2 and Ts + p kWY^2,
// column-major with leading dimension kb
__global__ void __launch_bounds__(kLP * kWY) k_larft(const double* __restrict__ Gs, const double* __restrict__ tau,
                                                     int n, double* __restrict__ Ts) {
  int j0, kb;
  panel(n, blockIdx.x, j0, kb);
  const double* G = Gs + (long long)blockIdx.x * kWY * kWY;
  double* T = Ts + (long long)blockIdx.x * kWY * kWY;
  // s[r][c]: T(r, c) on and above the diagonal, G(r, c) below it (G is symmetric)
  __shared__ double s[kWY][kWY + 1];
  __shared__ double tv[kWY];
  const int tid = threadIdx.x, i = tid / kLP, p = tid % kLP;
  for (int e = tid; e < kb * kb; e += kLP * kWY) {
    const int r = e % kb, c = e / kb;
    if (r > c) s[r][c] = G[e];
  }
  if (tid < kb) tv[tid] = tau[j0 + tid];
  if (p == i % kLP && i < kb) s[i][i] = tau[j0 + i];
  __syncthreads();
  // the wave's rows are i0 .. i0+15: its loop runs over the columns
  // k = p + kLP t with t from i0 / kLP (a multiple of 4) to the last one
  // below j, four at a time; partial sum q takes the columns with t = q
  // mod 4, in increasing t, so the sums do not depend on the wave
  const int i0 = __builtin_amdgcn_readfirstlane((tid >> 6) * (64 / kLP));
  for (int j = 1; j < kb; ++j) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    const int thi = (j + kLP - 1) / kLP;
    for (int t = i0 / kLP; t < thi; t += 4) {
      const int k0 = p + kLP * t, k1 = k0 + kLP, k2 = k1 + kLP, k3 = k2 + kLP;
      const bool u0 = k0 >= i && k0 < j, u1 = k1 >= i && k1 < j, u2 = k2 >= i && k2 < j, u3 = k3 >= i && k3 < j;
      const double r0 = s[i][u0 ? k0 : 0], r1 = s[i][u1 ? k1 : 0], r2 = s[i][u2 ? k2 : 0], r3 = s[i][u3 ? k3 : 0];
      const double g0 = s[j][u0 ? k0 : 0], g1 = s[j][u1 ? k1 : 0], g2 = s[j][u2 ? k2 : 0], g3 = s[j][u3 ? k3 : 0];
      a0 = fma(u0 ? r0 : 0.0, g0, a0);
      a1 = fma(u1 ? r1 : 0.0, g1, a1);
      a2 = fma(u2 ? r2 : 0.0, g2, a2);
      a3 = fma(u3 ? r3 : 0.0, g3, a3);
    }
    double acc = (a0 + a1) + (a2 + a3);
    acc += __shfl_xor(acc, 1, 64);  // the kLP = 4 parts of a row are adjacent lanes
    acc += __shfl_xor(acc, 2, 64);
    if (i < j && p == j % kLP) s[i][j] = -tv[j] * acc;
  }
  __syncthreads();
  for (int e = tid; e < kb * kb; e += kLP * kWY) {
    const int r = e % kb, c = e / kb;
    T[e] = r <= c ? s[r][c] : 0.0;
  }
}

// the products V^T Z and V^T V are short and wide (kWY rows of output over
// up to n rows of V): they run as a batch over row chunks of kSK rows, and the
// chunks' partial results are summed in a fixed order
constexpr int kSK = 256;
__global__ void __launch_bounds__(256) k_sumsplit(const double* __restrict__ parts, int nparts, long long len,
                                                  double* __restrict__ out) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= len) return;
  double acc = 0.0;
  for (int q = 0; q < nparts; ++q) acc += parts[(long long)q * len + e];
  out[e] = acc;
}

__global__ void k_tau_tail(double* tau, int n) {
  if (threadIdx.x == 0) tau[n - 2] = 0.0;
}

int cdiv(int a, int b) { return (a + b - 1) / b; }

}  // namespace

// workspace of the reduction: u (2 x n), y (n), z (n), s, and the partial
// sums py, pz (each ceil(n / 64) x n)
size_t gehrd_bytes(int n) {
  const size_t v = align_up(sizeof(double) * (size_t)n);
  return 4 * v + align_up(sizeof(double) * 8) + 2 * align_up(sizeof(double) * (size_t)n * cdiv(n, kT));
}

namespace {
// k_colhouse with the column in registers where it fits (n <= 8 kCH)
void colhouse(hipStream_t st, double* A, long long ld, int n, int q, double* tau, const double* uq, double* un,
              const double* y, const double* z, double* sc) {
  const int rows = cdiv(n, kCH);
  if (rows <= 1)
    hipLaunchKernelGGL(k_colhouse_r<1>, dim3(1), dim3(kCH), 0, st, A, ld, n, q, tau, uq, un, y, z, sc);
  else if (rows <= 2)
    hipLaunchKernelGGL(k_colhouse_r<2>, dim3(1), dim3(kCH), 0, st, A, ld, n, q, tau, uq, un, y, z, sc);
  else if (rows <= 4)
    hipLaunchKernelGGL(k_colhouse_r<4>, dim3(1), dim3(kCH), 0, st, A, ld, n, q, tau, uq, un, y, z, sc);
  else if (rows <= 8)
    hipLaunchKernelGGL(k_colhouse_r<8>, dim3(1), dim3(kCH), 0, st, A, ld, n, q, tau, uq, un, y, z, sc);
  else  // 16 rows per thread would spill at 128 registers per lane
    hipLaunchKernelGGL(k_colhouse, dim3(1), dim3(kCH), 0, st, A, ld, n, q, tau, uq, un, y, z, sc);
}
}  // namespace

int gehrd(hipStream_t st, int n, double* A, int lda, double* tau, void* work) {
  const size_t v = align_up(sizeof(double) * (size_t)n);
  double* u[2] = {static_cast<double*>(work), at<double>(work, v)};
  double* y = at<double>(work, 2 * v);
  double* z = at<double>(work, 3 * v);
  double* sc = at<double>(work, 4 * v);
  double* py = at<double>(work, 4 * v + align_up(sizeof(double) * 8));
  double* pz = py + (size_t)n * cdiv(n, kT);
  const long long ld = lda;
  const int nrt = cdiv(n, kT);
  if (n >= 3) {
    // the reflector of column 0 and the partial sums of step 0
    colhouse(st, A, ld, n, -1, tau, u[1], u[0], y, z, sc);
    hipLaunchKernelGGL((k_sweep<false, true, false>), dim3(nrt, cdiv(n - 1, kT)), dim3(256), 0, st, A, ld, n, -1, tau,
                       u[1], u[0], y, z, sc, py, pz);
    for (int q = 0; q <= n - 3; ++q) {
      const int m = n - q - 1;  // rows and columns q+1 .. n-1
      hipLaunchKernelGGL(k_reduce, dim3(cdiv(n + m, kRO)), dim3(kRO * kRG), 0, st, py, cdiv(m, kT), n, pz, nrt,
                         (long long)n, m, y, z);
      colhouse(st, A, ld, n, q, tau, u[q & 1], u[(q + 1) & 1], y, z, sc);
      const int nc = n - q - 2;  // columns q+2 .. n-1
      if (nc > 0) {
        const dim3 g(nrt, cdiv(nc, kT));
        // trailing columns larger than kNTBytes are read and written with
        // non-temporal hints (they are streamed once per step and do not
        // stay in the caches until the next step anyway)
        const bool nt = (double)sizeof(double) * n * nc > kNTBytes;
        if (q + 1 <= n - 3) {
          if (nt)
            hipLaunchKernelGGL((k_sweep<true, true, true>), g, dim3(256), 0, st, A, ld, n, q, tau, u[q & 1],
                               u[(q + 1) & 1], y, z, sc, py, pz);
          else
            hipLaunchKernelGGL((k_sweep<true, true, false>), g, dim3(256), 0, st, A, ld, n, q, tau, u[q & 1],
                               u[(q + 1) & 1], y, z, sc, py, pz);
        } else {
          hipLaunchKernelGGL((k_sweep<true, false, false>), g, dim3(256), 0, st, A, ld, n, q, tau, u[q & 1],
                             u[(q + 1) & 1], y, z, sc, py, pz);
        }
      }
    }
  }
  if (n >= 2) hipLaunchKernelGGL(k_tau_tail, dim3(1), dim3(64), 0, st, tau, n);
  return hipGetLastError() == hipSuccess ? HSRQ_OK : HSRQ_ERR_HIP;
}

// workspace of the back-transform: the panel V (n x kWY), G and T of every
// panel (kWY x kWY each), V^T Z and T V^T Z (kWY x ncols), and the chunk
// partials of V^T V and V^T Z
size_t ormhr_bytes(int n, int ncols) {
  const size_t nc = ncols > 0 ? ncols : 1;
  const size_t nsk = cdiv(n, kSK);
  const size_t np = npanels(n) > 0 ? npanels(n) : 1;
  return align_up(sizeof(double) * (size_t)n * kWY) + 2 * align_up(sizeof(double) * np * kWY * kWY) +
         2 * align_up(sizeof(double) * kWY * nc) + align_up(sizeof(double) * nsk * kWY * kWY) +
         align_up(sizeof(double) * nsk * kWY * nc);
}

namespace {
// C (kb x m) = V^T B over the nr rows of V (column-major, leading dimension
// nr) and of B (leading dimension ldb), as a batch over row chunks summed in
// order; P holds the chunk partials
bool gemm_tn_split(rocblas_handle bh, hipStream_t st, int kb, int m, int nr, const double* V, const double* B,
                   int ldb, double* P, double* C) {
  const double one = 1.0, zero = 0.0;
  const rocblas_operation tr = rocblas_operation_transpose, nt = rocblas_operation_none;
  const int full = nr / kSK, rem = nr - full * kSK;
  const long long len = (long long)kb * m;
  bool ok = true;
  if (full > 0)
    ok = rocblas_dgemm_strided_batched(bh, tr, nt, kb, m, kSK, &one, V, nr, kSK, B, ldb, kSK, &zero, P, kb, len,
                                       full) == rocblas_status_success;
  if (ok && rem > 0)
    ok = rocblas_dgemm(bh, tr, nt, kb, m, rem, &one, V + (long long)full * kSK, nr, B + (long long)full * kSK, ldb,
                       &zero, P + (long long)full * len, kb) == rocblas_status_success;
  const int nparts = full + (rem > 0 ? 1 : 0);
  hipLaunchKernelGGL(k_sumsplit, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, P, nparts, len, C);
  return ok;
}
}  // namespace

// Z <- Q0 Z = H_0 (H_1 ( ... (H_{n-3} Z))): panels of kWY reflectors from
// the last one down, each applied as Z(j0+1:n, :) -= V (T (V^T Z(j0+1:n, :)))
// with the products on rocBLAS (DGEMM on the handle's stream).  T depends on
// the reflectors alone, so a first pass forms G = V^T V of every panel and
// one launch builds every panel's T, one block per panel; the second pass
// applies the panels to Z.
int ormhr(hipStream_t st, void* blas, int n, const double* A, int lda, const double* tau, int ncols, double* Z,
          int ldz, void* work) {
  if (!blas) return HSRQ_ERR_HIP;
  rocblas_handle bh = static_cast<rocblas_handle>(blas);
  const size_t nsk = cdiv(n, kSK);
  const int np = npanels(n);
  const size_t npa = np > 0 ? np : 1;
  size_t off = 0;
  double* V = at<double>(work, off);
  off += align_up(sizeof(double) * (size_t)n * kWY);
  double* Gs = at<double>(work, off);
  off += align_up(sizeof(double) * npa * kWY * kWY);
  double* Ts = at<double>(work, off);
  off += align_up(sizeof(double) * npa * kWY * kWY);
  double* W = at<double>(work, off);
  off += align_up(sizeof(double) * kWY * (size_t)ncols);
  double* W2 = at<double>(work, off);
  off += align_up(sizeof(double) * kWY * (size_t)ncols);
  double* PG = at<double>(work, off);
  off += align_up(sizeof(double) * nsk * kWY * kWY);
  double* PW = at<double>(work, off);
  const double one = 1.0, zero = 0.0, mone = -1.0;
  const rocblas_operation nt = rocblas_operation_none;
  bool ok = true;
  for (int p = 0; p < np && ok; ++p) {  // G of every panel
    int j0, kb;
    panel(n, p, j0, kb);
    const int nr = n - (j0 + 1);
    hipLaunchKernelGGL(k_vpanel, dim3(cdiv(nr * kb, 256)), dim3(256), 0, st, A, (long long)lda, n, j0, kb, V);
    ok = gemm_tn_split(bh, st, kb, kb, nr, V, V, nr, PG, Gs + (size_t)p * kWY * kWY);
  }
  if (ok && np > 0) hipLaunchKernelGGL(k_larft, dim3(np), dim3(kLP * kWY), 0, st, Gs, tau, n, Ts);
  for (int p = 0; p < np && ok; ++p) {  // the panels applied to Z, the last one first
    int j0, kb;
    panel(n, p, j0, kb);
    const int nr = n - (j0 + 1);
    double* Zr = Z + (j0 + 1);
    const double* T = Ts + (size_t)p * kWY * kWY;
    hipLaunchKernelGGL(k_vpanel, dim3(cdiv(nr * kb, 256)), dim3(256), 0, st, A, (long long)lda, n, j0, kb, V);
    ok = ok && gemm_tn_split(bh, st, kb, ncols, nr, V, Zr, ldz, PW, W);
    ok = ok && rocblas_dgemm(bh, nt, nt, kb, ncols, kb, &one, T, kb, W, kb, &zero, W2, kb) == rocblas_status_success;
    ok = ok &&
         rocblas_dgemm(bh, nt, nt, nr, ncols, kb, &mone, V, nr, W2, kb, &one, Zr, ldz) == rocblas_status_success;
  }
  if (!ok) return HSRQ_ERR_HIP;
  return hipGetLastError() == hipSuccess ? HSRQ_OK : HSRQ_ERR_HIP;
}

}  // namespace hsrq

extern "C" {

int hsrq_gehrd_workspace_size(hsrq_handle_t h, int n, size_t* bytes) {
  if (!h) return -1;
  if (n < 1) return -2;
  if (!bytes) return -3;
  *bytes = hsrq::gehrd_bytes(n);
  return HSRQ_OK;
}

int hsrq_gehrd(hsrq_handle_t h, int n, double* A, int lda, double* tau, void* work, size_t work_bytes) {
  if (!h) return -1;
  if (n < 1) return -2;
  if (!A) return -3;
  if (lda < n) return -4;
  if (n >= 2 && !tau) return -5;
  if (!work || (reinterpret_cast<uintptr_t>(work) & 255) || work_bytes < hsrq::gehrd_bytes(n)) return -6;
  return hsrq::gehrd(hsrq::handle_stream(h), n, A, lda, tau, work);
}

int hsrq_ormhr_workspace_size(hsrq_handle_t h, int n, int ncols, size_t* bytes) {
  if (!h) return -1;
  if (n < 1) return -2;
  if (ncols < 0) return -3;
  if (!bytes) return -4;
  *bytes = hsrq::ormhr_bytes(n, ncols);
  return HSRQ_OK;
}

int hsrq_ormhr(hsrq_handle_t h, int n, const double* A, int lda, const double* tau, int ncols, double* Z, int ldz,
               void* work, size_t work_bytes) {
  if (!h) return -1;
  if (n < 1) return -2;
  if (!A) return -3;
  if (lda < n) return -4;
  if (n >= 2 && !tau) return -5;
  if (ncols < 0) return -6;
  if (ncols > 0 && !Z) return -7;
  if (ldz < n) return -8;
  if (!work || (reinterpret_cast<uintptr_t>(work) & 255) || work_bytes < hsrq::ormhr_bytes(n, ncols)) return -9;
  if (ncols == 0 || n < 3) return HSRQ_OK;
  return hsrq::ormhr(hsrq::handle_stream(h), hsrq::handle_blas(h), n, A, lda, tau, ncols, Z, ldz, work);
}

}  // extern "C"
