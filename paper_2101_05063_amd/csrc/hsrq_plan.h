// hsrq_plan.h -- host-side planning shared by the solve entry points and
// the serving loop: column layout, tiling, per-step task lists, workspace
// carving, and the kernel launch wrappers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "hsrq.h"
#include "hsrq_common.h"

namespace hsrq {

// nmax: the largest order among the nprob problems
void launch_prep(const ProbDesc* d, const int4* blk, int nblk, int nprob, int nmax, hipStream_t st);
void launch_init(const ProbDesc* d, const int4* blk, int nblk, hipStream_t st);
// allow the critical kernels their dynamic shared memory on the current
// device (0, or -1 on a HIP error); called once per handle and server
int crit_smem_init();
// share: the critical kernel variant that leaves room on its CU for one
// far-tile block (used for steps with at least share_min far-tile blocks of
// 64 columns, two blocks of 32 columns counting as one; kShareFar by
// default, opts.share_min_far otherwise)
constexpr int kShareFar = 512;
inline bool share_step(int nfar_blocks, int fcb, int share_min) {
  return (long long)nfar_blocks * fcb >= (long long)share_min * 64;
}
inline int share_min(const hsrq_opts_t* o) {
  if (!o || o->share_min_far == 0) return kShareFar;
  return o->share_min_far < 0 ? 0x7fffffff : o->share_min_far;
}
// cu: 1 = the variant that shares its CU with a far-tile block, 2 = the
// variant that takes the CU to itself (level-3 form at nb = 128: its block
// also claims the CU's free shared memory), 0 = the plain variant
void launch_crit(int nb, int prec, int l3rot, int cu, const ProbDesc* d, const Task* tasks, int ntasks,
                 hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// l3rot = 1 (and prec = 0): rotations of the off-diagonal cross-over columns
// applied as one product with the folded rotations W; else one at a time
// fcb: columns per far-tile block of the level-3 form (32 or 64; the
// one-at-a-time and FP32 forms always take 64)
void launch_far(int nb, int prec, int l3rot, int fcb, const ProbDesc* d, const Task* tasks, int ntasks,
                hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_final(const ProbDesc* d, const int2* cblk, int ncblk, const int4* fblk, int nfblk, hipStream_t st);
void launch_output(const ProbDesc* d, const int4* blk, int nblk, hipStream_t st);
void launch_resid(const ProbDesc* d, const int4* blk, int nblk, const int2* cblk, int ncblk, hipStream_t st);
// the sketched residual: skb lists (problem, 64-column tile of H), blk the
// (problem, 64-row block, column block) triples, cblk the column blocks
void launch_sketch(const ProbDesc* d, const int2* skb, int nskb, const int4* blk, int nblk, const int2* cblk,
                   int ncblk, hipStream_t st);
void launch_fill(double* p, long long cnt, double v, hipStream_t st);
void launch_copy(const CopyEnt* ents, int count, hipStream_t st);
void launch_gate(hipStream_t st);

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Layout {
  int ncols = 0;
  std::vector<int32_t> coltype, colshift, colsrc, colconj;
  std::vector<double> lr, li;
};

constexpr int kCrit = 8;    // columns of a critical task

struct ProbPlan {
  int n, N, nb, ncols, ld, nblk, nfblk;
  Layout lay;
  // byte offsets inside the workspace
  size_t o_meta_d, o_meta_i;              // head: lam_re, lam_im | 4 int arrays
  size_t o_V, o_X, o_Y, o_C, o_S, o_PHI, o_Z[2], o_W[2], o_BMAX, o_VMAX, o_BSSQ, o_BCMX, o_TN, o_FIN, o_AX, o_AMAX;
  size_t o_zero, o_HF, o_FLAG, o_HN, o_RPART, o_HFP, o_RNUMP, o_RK, o_SK, o_SKP;
};

struct Plan {
  int nb = 64;
  int fcb = 64;    // columns per far-tile block (b_c of the far tasks)
  int prec = 0;    // 1: FP32 tile-update products
  int l3rot = 0;   // 1: off-diagonal rotations folded and applied on MFMA (opts.rotations)
  int share = kShareFar;  // far-tile blocks from which a step uses the CU-sharing critical kernel
  int alone = 0;          // 1: the other steps' critical kernel takes its CU to itself (see launch_crit)
  std::vector<ProbPlan> pp;
  std::vector<Task> tasks;
  std::vector<int> coff, ccnt, foff, fcnt;  // per step: critical and far task ranges
  std::vector<int2> blk_cols;
  std::vector<int4> blk_prep, blk_init, blk_out, blk_fin;
  std::vector<int2> blk_skh;  // (problem, 64-column tile of H): the sketch of H
  size_t o_desc, o_tasks, o_bprep, o_bcols, o_binit, o_bout, o_bfin, o_bskh;
  size_t head_bytes, total_bytes;
  size_t o_zero_all = 0, zero_count = 0;  // doubles
  int nmax = 0;                           // largest order
};

// Carve the workspace and build every host-side table.
// Complex shifts first as aligned [re im] pairs, then real shifts, each group
// in the caller's order (the real/complex split of Algorithm 15).
Layout make_layout(int m, const double* wr, const double* wi);
int count_cols(int m, const double* wi);
// Carve the workspace and build every host-side table for tile size nb.
// fcb: columns per far-tile block (64, or 32 for the level-3 form)
void build_plan(Plan& P, int count, const hsrq_problem_t* probs, int nb, int fcb = 64);
// Writes the plan's head region (descriptors, task and block tables, column
// metadata) into the host image hb.
void fill_staging(const Plan& P, int count, const hsrq_problem_t* probs, void* work, const hsrq_opts_t* o,
                  char* hb);
// 0, or -k for an invalid k-th argument of the single-problem call
int check_problem(const hsrq_problem_t& p);
// options outside their documented values
bool opts_valid(const hsrq_opts_t* o);

// scratch for hsrq_dhsrq3_noalloc (hsrq_noalloc.hip): scratch_init records
// the address of the device's copy (once per device, with it current)
int scratch_init(int device);
int handle_device(hsrq_handle_t h);
hipStream_t handle_stream(hsrq_handle_t h);
// the handle's rocBLAS handle (a rocblas_handle, created on first use, on
// the handle's stream); null if rocBLAS could not create it
void* handle_blas(hsrq_handle_t h);
int run_noalloc(hsrq_handle_t h, const hsrq_problem_t& p, void* work, size_t work_bytes, const hsrq_opts_t* o);

template <class T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

}  // namespace hsrq
