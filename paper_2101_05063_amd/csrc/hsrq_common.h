// hsrq_common.h -- shared definitions of the HIP library (device and host).
//
// Internal data layout (one problem of order n with ncols internal columns):
//   * columns are reordered so that every complex shift occupies an aligned
//     pair [re im] (complex shifts first, then real ones); a shift with a
//     negative imaginary part is replaced by its conjugate (Sec. 4.3: one
//     member per conjugate pair) and the result conjugated back;
//   * vector arrays (working columns V, right-hand sides / solutions X,
//     rotations C, S and diagonal PHI) are row-major n x ld, so that the 64
//     lanes of a wave that own 64 consecutive columns touch one contiguous
//     512-byte row segment;
//   * tiles are aligned to the bottom-right corner of H: tile t (0-based)
//     covers rows/columns [tstart(t), tend(t)), tend(t) = n - (N-1-t) nb, so
//     only the top-left tile can be ragged (Sec. 3.2 assumes n = N b_r).
#pragma once
#include <stdint.h>

namespace hsrq {

constexpr int kTExp = 1000;        // stored magnitudes stay below 2^kTExp
constexpr int kNegExp = -100000;   // exponent of zero
constexpr int kSingExp = 1 << 29;  // segment exponent of an exactly singular R(1,1)
constexpr int kCB = 64;            // columns per block (shifts-per-block b_c, in columns)
constexpr int kChunk = 32;         // rows per chunk of the final scan (host tables and kernels)

enum ColType : int32_t { CT_REAL = 0, CT_CRE = 1, CT_CIM = 2 };
enum TaskType : int32_t { TK_CHAIN = 0, TK_CRIT = 1, TK_FAR = 2 };
enum FlagBits : int32_t { FL_NONFINITE = 1, FL_REDUCED = 2 };

struct ProbDesc {
  const double* H;
  long long ldh;
  int n, N, nb, ncols, ld, nblk, nfblk, m, precision;  // nfblk: far-tile column blocks
  // workspace (device)
  double *V, *X, *Y, *C, *S, *PHI;
  // Z and W panels, two per problem: the critical task of step t writes
  // slot t & 1 and the tasks of step t + 1 read it (every task of step t + 1
  // has finished before step t + 2 writes the slot again)
  double* Z[2];
  double* W[2];
  double *BMAX, *VMAX, *BSSQ, *BCMX, *TN, *FIN;
  int32_t *AX, *AMAX;
  // partial sums written once per call and reduced in a fixed order, so that
  // every norm is the same on every run: row sums of |h| per (row, tile
  // column) RPART[jt * n + row], sums of h^2 per tile pair HFP[i * N + jt],
  // residual sums of squares per (64-row block, column) RNUMP[rb * ld + col]
  double *RPART, *HFP, *RNUMP;
  // sketched residual (mixed precision's check): probe entries RK[k * n + i],
  // the sketch of H SK[k * n + j] = sum_i RK[k][i] h(i, j), and per 64-row
  // block the partial sums SKP[(rb * 16 + q) * ld + col] of RK y (q < 8) and
  // SK y (q >= 8)
  double *RK, *SK, *SKP;
  // zero-initialised per call: ||H||_F^2 (written by the reduction), flags,
  // ||H||_inf (a maximum of non-negative doubles, taken on their bit patterns)
  double* HF;
  int32_t* FLAG;
  double* HN;
  // column metadata (device)
  const double *lam_re, *lam_im;
  const int32_t *coltype, *colshift, *colsrc, *colconj;
  // caller outputs (device)
  double* Xu;
  long long ldx;
  int32_t* Eu;
  double* Mu;
  int32_t* Iu;
  double* Ru;
};

// one block of a step launch: problem, task type | (step << 8), tile row,
// column block.  The step travels with the task so that one launch can hold
// problems at different steps (continuous batching).
struct Task {
  int32_t prob, type, i, L;
};
__host__ __device__ inline int32_t task_code(int type, int step) { return type | (step << 8); }
__host__ __device__ inline int task_type(int32_t code) { return code & 0xff; }
__host__ __device__ inline int task_step(int32_t code) { return code >> 8; }

// one copy of a gather/scatter list (bytes, a multiple of 4)
struct CopyEnt {
  const void* src;
  void* dst;
  long long nbytes;
};

// the Z / W panel slot written by the critical task of step t
__host__ __device__ inline int zw_slot(int t) { return t & 1; }

__host__ __device__ inline int tile_end(int n, int N, int nb, int t) { return n - (N - 1 - t) * nb; }
__host__ __device__ inline int tile_start(int n, int N, int nb, int t) {
  int e = tile_end(n, N, nb, t);
  return e - nb > 0 ? e - nb : 0;
}
__host__ __device__ inline int tile_of_row(int n, int N, int nb, int r) {
  return N - 1 - (n - 1 - r) / nb;
}

}  // namespace hsrq
