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
// One Householder step per column, on the device:
//   k_house        the reflector of column k (one block; norms by a scaled
//                  sum of squares reduced in a fixed order)
//   k_gemv_rows    y = A(:, k+1:n) u, partial sums per column chunk, and
//   k_sum_chunks   their sum in chunk order
//   k_rank1        A(r0:, c0:) -= tau y u^T (from the right) or
//                  tau u w^T (from the left), 64 x 64 tiles
//   k_dot_cols     w = u^T A(k+1:n, k+1:n): one wave per column
// (right application first, then left, as LAPACK's DGEHD2).  The
// back-transform applies the reflectors in reverse order to the columns of
// Z with k_dot_cols and k_rank1.  Every reduction has a fixed order, so the
// results are the same on every run.
#include <hip/hip_runtime.h>
#include <math.h>

#include "hsrq.h"
#include "hsrq_plan.h"

namespace hsrq {
namespace {

constexpr int kChunkCols = 256;  // columns per partial sum of k_gemv_rows

__device__ __forceinline__ double wsum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ double wmax(double x) {
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

// Reflector of column k: x = A(k+1:n, k), m = n-k-1 entries.  Writes beta to
// A(k+1, k), v = x(2:m) / (alpha - beta) in place, tau[k], and u = [1; v]
// (length m) to the workspace.  One block of 1024 threads.
__global__ void __launch_bounds__(1024) k_house(double* A, long long lda, int n, int k, double* tau, double* u) {
  const int m = n - k - 1;
  double* x = A + (k + 1) + (long long)k * lda;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  __shared__ double red[16];
  __shared__ double bc[3];
  double mx = 0.0;
  for (int i = 1 + tid; i < m; i += 1024) mx = fmax(mx, fabs(x[i]));
  mx = wmax(mx);
  if (lane == 0) red[w] = mx;
  __syncthreads();
  if (tid == 0) {
    double v = 0.0;
    for (int j = 0; j < 16; ++j) v = fmax(v, red[j]);
    bc[0] = v;
  }
  __syncthreads();
  mx = bc[0];
  double ss = 0.0;
  if (mx > 0.0)
    for (int i = 1 + tid; i < m; i += 1024) {
      const double t = x[i] / mx;
      ss = fma(t, t, ss);
    }
  ss = wsum(ss);
  __syncthreads();
  if (lane == 0) red[w] = ss;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int j = 0; j < 16; ++j) s += red[j];
    const double xnorm = mx * sqrt(s);
    const double alpha = x[0];
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
    tau[k] = t;
    bc[1] = beta;
    bc[2] = scal;
  }
  __syncthreads();
  const double scal = bc[2];
  for (int i = 1 + tid; i < m; i += 1024) {
    const double v = x[i] * scal;
    x[i] = v;
    u[i] = v;
  }
  if (tid == 0) {
    x[0] = bc[1];
    u[0] = 1.0;
  }
}

// partial[chunk][r] = sum over the chunk's columns c of A(r, c0 + c) u[c],
// rows r < nr; block = 64 rows x 4 column phases
__global__ void __launch_bounds__(256) k_gemv_rows(const double* A, long long lda, int nr, int c0, int nc,
                                                   const double* u, double* partial) {
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int r = blockIdx.x * 64 + tx;
  const int ch = blockIdx.y;
  const int cb = ch * kChunkCols, ce = min(nc, cb + kChunkCols);
  __shared__ double red[4][64];
  double s = 0.0;
  if (r < nr)
    for (int c = cb + ty; c < ce; c += 4) s = fma(A[r + (long long)(c0 + c) * lda], u[c], s);
  red[ty][tx] = s;
  __syncthreads();
  if (ty == 0 && r < nr) partial[(long long)ch * nr + r] = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
}

__global__ void __launch_bounds__(256) k_sum_chunks(const double* partial, int nr, int nch, double* y) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= nr) return;
  double s = 0.0;
  for (int ch = 0; ch < nch; ++ch) s += partial[(long long)ch * nr + r];
  y[r] = s;
}

// w[c] = sum_r u[r] M(r0 + r, c0 + c), r < nr: one wave per column
__global__ void __launch_bounds__(256) k_dot_cols(const double* M, long long ldm, int r0, int nr, int c0, int nc,
                                                  const double* u, double* w) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (c >= nc) return;
  const double* col = M + r0 + (long long)(c0 + c) * ldm;
  double s = 0.0;
  for (int r = lane; r < nr; r += 64) s = fma(u[r], col[r], s);
  s = wsum(s);
  if (lane == 0) w[c] = s;
}

// M(r0 + r, c0 + c) -= tau[k] a[r] b[c] over nr x nc, 64 x 64 tiles
__global__ void __launch_bounds__(256) k_rank1(double* M, long long ldm, int r0, int nr, int c0, int nc,
                                               const double* tau, int k, const double* a, const double* b) {
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int r = blockIdx.x * 64 + tx;
  const double t = tau[k];
  if (r >= nr || t == 0.0) return;
  const double ar = t * a[r];
  for (int cc = ty; cc < 64; cc += 4) {
    const int c = blockIdx.y * 64 + cc;
    if (c < nc) {
      double* p = M + r0 + r + (long long)(c0 + c) * ldm;
      *p = fma(-ar, b[c], *p);
    }
  }
}

// tau[n-2] = 0: the last reflector is the identity (LAPACK's convention)
__global__ void k_tau_tail(double* tau, int n) {
  if (threadIdx.x == 0) tau[n - 2] = 0.0;
}

// u = [1; A(k+2:n, k)] (the stored reflector of column k), m = n-k-1 entries
__global__ void __launch_bounds__(256) k_make_u(const double* A, long long lda, int n, int k, double* u) {
  const int i = blockIdx.x * 256 + threadIdx.x, m = n - k - 1;
  if (i < m) u[i] = i == 0 ? 1.0 : A[(k + 1 + i) + (long long)k * lda];
}

dim3 tiles(int nr, int nc) { return dim3((nr + 63) / 64, (nc + 63) / 64); }

}  // namespace

// workspace of the reduction: u (n), y (n), w (n), partial sums
size_t gehrd_bytes(int n) {
  const int nch = (n + kChunkCols - 1) / kChunkCols;
  return align_up(sizeof(double) * (size_t)n) * 3 + align_up(sizeof(double) * (size_t)n * nch);
}

int gehrd(hipStream_t st, int n, double* A, int lda, double* tau, void* work) {
  double* u = static_cast<double*>(work);
  double* y = at<double>(work, align_up(sizeof(double) * (size_t)n));
  double* w = at<double>(work, 2 * align_up(sizeof(double) * (size_t)n));
  double* part = at<double>(work, 3 * align_up(sizeof(double) * (size_t)n));
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // rows and columns k+1 .. n-1
    hipLaunchKernelGGL(k_house, dim3(1), dim3(1024), 0, st, A, (long long)lda, n, k, tau, u);
    // from the right: A(0:n, k+1:n) -= tau (A(0:n, k+1:n) u) u^T
    const int nch = (m + kChunkCols - 1) / kChunkCols;
    hipLaunchKernelGGL(k_gemv_rows, dim3((n + 63) / 64, nch), dim3(256), 0, st, A, (long long)lda, n, k + 1, m, u,
                       part);
    hipLaunchKernelGGL(k_sum_chunks, dim3((n + 255) / 256), dim3(256), 0, st, part, n, nch, y);
    hipLaunchKernelGGL(k_rank1, tiles(n, m), dim3(256), 0, st, A, (long long)lda, 0, n, k + 1, m, tau, k, y, u);
    // from the left: A(k+1:n, k+1:n) -= tau u (u^T A(k+1:n, k+1:n))
    hipLaunchKernelGGL(k_dot_cols, dim3((m + 3) / 4), dim3(256), 0, st, A, (long long)lda, k + 1, m, k + 1, m, u, w);
    hipLaunchKernelGGL(k_rank1, tiles(m, m), dim3(256), 0, st, A, (long long)lda, k + 1, m, k + 1, m, tau, k, u, w);
  }
  if (n >= 2) hipLaunchKernelGGL(k_tau_tail, dim3(1), dim3(64), 0, st, tau, n);
  return hipGetLastError() == hipSuccess ? HSRQ_OK : HSRQ_ERR_HIP;
}

// workspace of the back-transform: u (n), w (ncols)
size_t ormhr_bytes(int n, int ncols) {
  return align_up(sizeof(double) * (size_t)n) + align_up(sizeof(double) * (size_t)(ncols > 0 ? ncols : 1));
}

// Z <- Q0 Z = H_0 (H_1 ( ... (H_{n-3} Z)))
int ormhr(hipStream_t st, int n, const double* A, int lda, const double* tau, int ncols, double* Z, int ldz,
          void* work) {
  double* u = static_cast<double*>(work);
  double* w = at<double>(work, align_up(sizeof(double) * (size_t)n));
  for (int k = n - 3; k >= 0; --k) {
    const int m = n - k - 1;
    hipLaunchKernelGGL(k_make_u, dim3((m + 255) / 256), dim3(256), 0, st, A, (long long)lda, n, k, u);
    hipLaunchKernelGGL(k_dot_cols, dim3((ncols + 3) / 4), dim3(256), 0, st, Z, (long long)ldz, k + 1, m, 0, ncols, u,
                       w);
    hipLaunchKernelGGL(k_rank1, tiles(m, ncols), dim3(256), 0, st, Z, (long long)ldz, k + 1, m, 0, ncols, tau, k, u,
                       w);
  }
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
  return hsrq::ormhr(hsrq::handle_stream(h), n, A, lda, tau, ncols, Z, ldz, work);
}

}  // extern "C"
