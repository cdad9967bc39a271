// hsrq_host.cpp -- C-ABI entry points, planning and launch sequence.
//
// A call plans on the host (column layout, tiling, per-step task lists,
// workspace carving), copies the plan into the head of the caller's device
// workspace with one asynchronous copy from a pinned staging buffer, and
// enqueues the kernels on the handle's stream.  Nothing is allocated on the
// device inside a solve.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "hsrq.h"
#include "hsrq_common.h"
#include "hsrq_plan.h"


using namespace hsrq;

namespace hsrq {

Layout make_layout(int m, const double* wr, const double* wi) {
  Layout L;
  std::vector<int> ccol(m);
  int c = 0;
  for (int l = 0; l < m; ++l) {
    ccol[l] = c;
    c += (wi && wi[l] != 0.0) ? 2 : 1;
  }
  auto push = [&](int type, int shift, int src, int conj, double r, double i) {
    L.coltype.push_back(type);
    L.colshift.push_back(shift);
    L.colsrc.push_back(src);
    L.colconj.push_back(conj);
    L.lr.push_back(r);
    L.li.push_back(i);
  };
  for (int l = 0; l < m; ++l) {
    if (!(wi && wi[l] != 0.0)) continue;
    const bool bad = !std::isfinite(wr[l]) || !std::isfinite(wi[l]);
    const int conj = (wi[l] < 0.0 ? 1 : 0) | (bad ? 2 : 0);
    const double r = bad ? 0.0 : wr[l], i = bad ? 1.0 : std::fabs(wi[l]);
    push(CT_CRE, l, ccol[l], conj, r, i);
    push(CT_CIM, l, ccol[l] + 1, conj, r, i);
  }
  for (int l = 0; l < m; ++l) {
    if (wi && wi[l] != 0.0) continue;
    const bool bad = !std::isfinite(wr[l]) || (wi && !std::isfinite(wi[l]));
    push(CT_REAL, l, ccol[l], bad ? 2 : 0, bad ? 0.0 : wr[l], 0.0);
  }
  L.ncols = (int)L.coltype.size();
  return L;
}

int count_cols(int m, const double* wi) {
  int c = 0;
  for (int l = 0; l < m; ++l) c += (wi[l] != 0.0) ? 2 : 1;
  return c;
}

// Workgroups of a launch go to the 8 XCDs of the device in turn (workgroup b
// to XCD b % 8), and each XCD has its own L2.  Reorder a task list so that
// XCD x receives a contiguous run of it: the column blocks of one tile row,
// which share the H tile, then land on one XCD (two at a run boundary).
constexpr int kXcds = 8;
void xcd_order(Task* t, int n) {
  if (n <= kXcds) return;
  std::vector<Task> src(t, t + n);
  int start = 0;
  for (int x = 0; x < kXcds; ++x) {
    const int cnt = (n - x + kXcds - 1) / kXcds;  // workgroups b < n with b % 8 == x
    for (int j = 0; j < cnt; ++j) t[x + kXcds * j] = src[start + j];
    start += cnt;
  }
}

void build_plan(Plan& P, int count, const hsrq_problem_t* probs, int nb_choice, int fcb) {
  P.nb = nb_choice;
  P.fcb = fcb;
  P.alone = count == 1 ? 1 : 0;
  const int nb = P.nb;
  P.pp.resize(count);
  int Tmax = 0;
  for (int p = 0; p < count; ++p) {
    ProbPlan& q = P.pp[p];
    q.n = probs[p].n;
    q.nb = nb;
    q.N = (q.n + nb - 1) / nb;
    q.lay = make_layout(probs[p].m, probs[p].wr, probs[p].wi);
    q.ncols = q.lay.ncols;
    // the rows of the row-major workspace arrays (X, V, ...) start on
    // 128-byte cache lines, so that a block's row segment is whole lines
    q.ld = std::max(16, (q.ncols + 15) & ~15);
    q.nblk = (q.ncols + kCB - 1) / kCB;
    q.nfblk = (q.ncols + fcb - 1) / fcb;
    if (q.ncols > 0) Tmax = std::max(Tmax, q.N);
    P.nmax = std::max(P.nmax, q.n);
  }
  // tasks: step t = 0 chains the last tile; step t >= 1 works on tile column
  // jt = N - t (critical tasks first, then far tasks)
  P.coff.assign(Tmax, 0);
  P.ccnt.assign(Tmax, 0);
  P.foff.assign(Tmax, 0);
  P.fcnt.assign(Tmax, 0);
  for (int t = 0; t < Tmax; ++t) {
    P.coff[t] = (int)P.tasks.size();
    for (int p = 0; p < count; ++p) {
      const ProbPlan& q = P.pp[p];
      if (q.ncols == 0 || q.N <= t) continue;
      const int ncrit = (q.ncols + kCrit - 1) / kCrit;
      for (int L = 0; L < ncrit; ++L) {
        if (t == 0)
          P.tasks.push_back(Task{p, task_code(TK_CHAIN, 0), q.N - 1, L});
        else
          P.tasks.push_back(Task{p, task_code(TK_CRIT, t), q.N - t - 1, L});
      }
    }
    P.ccnt[t] = (int)P.tasks.size() - P.coff[t];
    P.foff[t] = (int)P.tasks.size();
    if (t > 0) {
      for (int p = 0; p < count; ++p) {
        const ProbPlan& q = P.pp[p];
        if (q.ncols == 0 || q.N <= t) continue;
        const int jt = q.N - t;
        for (int i = 0; i < jt - 1; ++i)
          for (int L = 0; L < q.nfblk; ++L) P.tasks.push_back(Task{p, task_code(TK_FAR, t), i, L});
      }
    }
    P.fcnt[t] = (int)P.tasks.size() - P.foff[t];
    xcd_order(P.tasks.data() + P.foff[t], P.fcnt[t]);
  }
  for (int p = 0; p < count; ++p) {
    const ProbPlan& q = P.pp[p];
    if (q.ncols == 0) continue;
    for (int t = 0; t < q.N; ++t) {
      for (int jt = t; jt < q.N; ++jt) P.blk_prep.push_back(int4{p, t, jt, 0});
      for (int L = 0; L < q.nblk; ++L) P.blk_init.push_back(int4{p, t, L, 0});
    }
    for (int L = 0; L < q.nblk; ++L) P.blk_cols.push_back(int2{p, L});
    for (int r = 0; r < (q.n + 63) / 64; ++r)
      for (int L = 0; L < q.nblk; ++L) P.blk_out.push_back(int4{p, r, L, 0});
    for (int j = 0; j < (q.n + 63) / 64; ++j) P.blk_skh.push_back(int2{p, j});
    const int nch = (q.n + kChunk - 1) / kChunk;
    for (int g = 0; g < (nch + 3) / 4; ++g)
      for (int L = 0; L < q.nblk; ++L) P.blk_fin.push_back(int4{p, g, L, 0});
  }
  // head: descriptors, tables, column metadata
  size_t off = 0;
  P.o_desc = off; off = align_up(off + sizeof(ProbDesc) * std::max(count, 1));
  P.o_tasks = off; off = align_up(off + sizeof(Task) * std::max<size_t>(P.tasks.size(), 1));
  P.o_bprep = off; off = align_up(off + sizeof(int4) * std::max<size_t>(P.blk_prep.size(), 1));
  P.o_bcols = off; off = align_up(off + sizeof(int2) * std::max<size_t>(P.blk_cols.size(), 1));
  P.o_binit = off; off = align_up(off + sizeof(int4) * std::max<size_t>(P.blk_init.size(), 1));
  P.o_bout = off; off = align_up(off + sizeof(int4) * std::max<size_t>(P.blk_out.size(), 1));
  P.o_bfin = off; off = align_up(off + sizeof(int4) * std::max<size_t>(P.blk_fin.size(), 1));
  P.o_bskh = off; off = align_up(off + sizeof(int2) * std::max<size_t>(P.blk_skh.size(), 1));
  for (auto& q : P.pp) {
    q.o_meta_d = off; off = align_up(off + sizeof(double) * 2 * q.ld);
    q.o_meta_i = off; off = align_up(off + sizeof(int32_t) * 4 * q.ld);
  }
  P.head_bytes = off;
  // zero-initialised scalars of every problem, contiguous for one fill:
  // ||H||_F^2 (1), flags (1 slot), ||H||_inf (1)
  P.o_zero_all = off;
  for (auto& q : P.pp) {
    q.o_zero = off;
    q.o_HF = off; off += sizeof(double);
    q.o_FLAG = off; off += sizeof(double);
    q.o_HN = off; off += sizeof(double);
  }
  P.zero_count = (off - P.o_zero_all) / sizeof(double);
  off = align_up(off);
  for (auto& q : P.pp) {
    const size_t vec = sizeof(double) * (size_t)q.n * q.ld;
    q.o_V = off; off = align_up(off + vec);
    q.o_X = off; off = align_up(off + vec);
    q.o_Y = off; off = align_up(off + vec);
    q.o_C = off; off = align_up(off + vec);
    q.o_S = off; off = align_up(off + vec);
    q.o_PHI = off; off = align_up(off + vec);
    for (int k = 0; k < 2; ++k) {
      q.o_Z[k] = off; off = align_up(off + sizeof(double) * (size_t)(nb + 3) * q.ld);
      q.o_W[k] = off; off = align_up(off + sizeof(double) * (size_t)(nb + 1) * q.ld);
    }
    q.o_BMAX = off; off = align_up(off + sizeof(double) * (size_t)q.N * q.ld);
    q.o_VMAX = off; off = align_up(off + sizeof(double) * (size_t)q.N * q.ld);
    q.o_BSSQ = off; off = align_up(off + sizeof(double) * (size_t)q.N * q.ld);
    q.o_BCMX = off; off = align_up(off + sizeof(double) * (size_t)q.N * q.ld);
    q.o_AX = off; off = align_up(off + sizeof(int32_t) * (size_t)q.N * q.ld);
    q.o_AMAX = off; off = align_up(off + sizeof(int32_t) * q.ld);
    q.o_TN = off; off = align_up(off + sizeof(double) * (size_t)q.N * q.N);
    q.o_RPART = off; off = align_up(off + sizeof(double) * (size_t)q.N * q.n);
    q.o_HFP = off; off = align_up(off + sizeof(double) * (size_t)q.N * q.N);
    q.o_RNUMP = off; off = align_up(off + sizeof(double) * (size_t)((q.n + 63) / 64) * q.ld);
    q.o_RK = off; off = align_up(off + sizeof(double) * 8 * (size_t)q.n);
    q.o_SK = off; off = align_up(off + sizeof(double) * 8 * (size_t)q.n);
    q.o_SKP = off; off = align_up(off + sizeof(double) * 16 * (size_t)((q.n + 511) / 512) * q.ld);
    const size_t nch = (q.n + kChunk - 1) / kChunk;
    q.o_FIN = off; off = align_up(off + sizeof(double) * (nch * 8 + 1) * q.ld);
  }
  P.total_bytes = off;
}

// Writes the plan's head region (descriptors, task and block tables, column
// metadata) into the host image hb.
void fill_staging(const Plan& P, int count, const hsrq_problem_t* probs, void* work, const hsrq_opts_t* o,
                  char* hb) {
  std::memset(hb, 0, P.head_bytes);
  std::vector<ProbDesc> descs(count);
  for (int p = 0; p < count; ++p) {
    const ProbPlan& q = P.pp[p];
    const hsrq_problem_t& pr = probs[p];
    ProbDesc& d = descs[p];
    std::memset(&d, 0, sizeof(d));
    d.H = pr.H;
    d.ldh = pr.ldh;
    d.n = q.n; d.N = q.N; d.nb = q.nb; d.ncols = q.ncols; d.ld = q.ld; d.nblk = q.nblk; d.nfblk = q.nfblk; d.m = pr.m;
    d.precision = o ? o->precision : 0;
    d.V = at<double>(work, q.o_V);
    d.X = at<double>(work, q.o_X);
    d.Y = at<double>(work, q.o_Y);
    d.C = at<double>(work, q.o_C);
    d.S = at<double>(work, q.o_S);
    d.PHI = at<double>(work, q.o_PHI);
    for (int k = 0; k < 2; ++k) {
      d.Z[k] = at<double>(work, q.o_Z[k]);
      d.W[k] = at<double>(work, q.o_W[k]);
    }
    d.BMAX = at<double>(work, q.o_BMAX);
    d.VMAX = at<double>(work, q.o_VMAX);
    d.BSSQ = at<double>(work, q.o_BSSQ);
    d.BCMX = at<double>(work, q.o_BCMX);
    d.TN = at<double>(work, q.o_TN);
    d.FIN = at<double>(work, q.o_FIN);
    d.AX = at<int32_t>(work, q.o_AX);
    d.AMAX = at<int32_t>(work, q.o_AMAX);
    d.RPART = at<double>(work, q.o_RPART);
    d.HFP = at<double>(work, q.o_HFP);
    d.RNUMP = at<double>(work, q.o_RNUMP);
    d.RK = at<double>(work, q.o_RK);
    d.SK = at<double>(work, q.o_SK);
    d.SKP = at<double>(work, q.o_SKP);
    d.HF = at<double>(work, q.o_HF);
    d.FLAG = at<int32_t>(work, q.o_FLAG);
    d.HN = at<double>(work, q.o_HN);
    d.lam_re = at<double>(work, q.o_meta_d);
    d.lam_im = at<double>(work, q.o_meta_d) + q.ld;
    d.coltype = at<int32_t>(work, q.o_meta_i);
    d.colshift = at<int32_t>(work, q.o_meta_i) + q.ld;
    d.colsrc = at<int32_t>(work, q.o_meta_i) + 2 * q.ld;
    d.colconj = at<int32_t>(work, q.o_meta_i) + 3 * q.ld;
    d.Xu = pr.X;
    d.ldx = pr.ldx;
    d.Eu = pr.scale_exp;
    d.Mu = pr.scale_mant;
    d.Iu = pr.info;
    d.Ru = pr.resid;
    double* md = reinterpret_cast<double*>(hb + q.o_meta_d);
    int32_t* mi = reinterpret_cast<int32_t*>(hb + q.o_meta_i);
    for (int c = 0; c < q.ncols; ++c) {
      md[c] = q.lay.lr[c];
      md[q.ld + c] = q.lay.li[c];
      mi[c] = q.lay.coltype[c];
      mi[q.ld + c] = q.lay.colshift[c];
      mi[2 * q.ld + c] = q.lay.colsrc[c];
      mi[3 * q.ld + c] = q.lay.colconj[c];
    }
  }
  std::memcpy(hb + P.o_desc, descs.data(), sizeof(ProbDesc) * count);
  if (!P.tasks.empty()) std::memcpy(hb + P.o_tasks, P.tasks.data(), sizeof(Task) * P.tasks.size());
  if (!P.blk_prep.empty()) std::memcpy(hb + P.o_bprep, P.blk_prep.data(), sizeof(int4) * P.blk_prep.size());
  if (!P.blk_fin.empty()) std::memcpy(hb + P.o_bfin, P.blk_fin.data(), sizeof(int4) * P.blk_fin.size());
  if (!P.blk_cols.empty()) std::memcpy(hb + P.o_bcols, P.blk_cols.data(), sizeof(int2) * P.blk_cols.size());
  if (!P.blk_init.empty()) std::memcpy(hb + P.o_binit, P.blk_init.data(), sizeof(int4) * P.blk_init.size());
  if (!P.blk_out.empty()) std::memcpy(hb + P.o_bout, P.blk_out.data(), sizeof(int4) * P.blk_out.size());
  if (!P.blk_skh.empty()) std::memcpy(hb + P.o_bskh, P.blk_skh.data(), sizeof(int2) * P.blk_skh.size());
}

int check_problem(const hsrq_problem_t& p) {
  if (p.n < 1) return -2;
  if (!p.H) return -3;
  if (p.ldh < p.n) return -4;
  if (p.m < 0) return -5;
  if (p.m > 0 && !p.wr) return -6;
  if (p.m > 0 && !p.wi) return -7;
  if (p.m > 0 && !p.X) return -8;
  if (p.ldx < p.n) return -9;
  if (p.m > 0 && !p.scale_exp) return -10;
  if (p.m > 0 && !p.scale_mant) return -11;
  if (p.m > 0 && !p.info) return -12;
  return 0;
}

}  // namespace hsrq


struct hsrq_handle_s {
  int device = 0;
  hipStream_t stream = nullptr;
  void* staging = nullptr;
  size_t staging_bytes = 0;
  hipEvent_t staging_ev = nullptr;
  bool staging_pending = false;
  // second stream for the far-tile kernels, and fork/join events
  hipStream_t aux = nullptr;
  // fork, critical step done, far step done: each wait is enqueued before the
  // event is recorded again, and a wait refers to the record preceding it
  hipEvent_t sync_ev[3] = {nullptr, nullptr, nullptr};
  // profiling
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used;
  // graph replay: a capture stream and a small cache of instantiated launch
  // sequences, each with two pinned staging buffers used alternately
  hipStream_t cap = nullptr;
  struct GraphSlot {
    hipGraphExec_t exec = nullptr;
    void* staging = nullptr;
    hipEvent_t done = nullptr;
    bool pending = false;
  };
  struct GraphEntry {
    uint64_t key = 0;
    uint64_t stamp = 0;
    size_t head_bytes = 0;
    GraphSlot slot[2];
    int next = 0;
  };
  std::vector<GraphEntry> graphs;
  uint64_t stamp = 0;
  // autotuner results: problem-set signature -> tile size, far-block width
  struct Tuned {
    uint64_t key;
    int nb, fcb;
  };
  std::vector<Tuned> tuned;
  // mixed precision: shifts re-solved in FP64 by the last call, and a pinned
  // buffer for the gather/scatter lists (read by the copy kernel in place)
  size_t last_fallback = 0;
  void* lists = nullptr;
  size_t lists_bytes = 0;
  hipEvent_t lists_ev = nullptr;
  bool lists_pending = false;
  // rocBLAS handle of the blocked back-transform (created on first use)
  rocblas_handle blas = nullptr;
};

namespace {

constexpr int kNbCandidates[2] = {64, 128};

// FNV-1a over 64-bit words
struct Sig {
  uint64_t v = 1469598103934665603ull;
  void add(uint64_t x) {
    for (int b = 0; b < 8; ++b) {
      v ^= (x >> (8 * b)) & 0xff;
      v *= 1099511628211ull;
    }
  }
};

// the autotuner's key: orders and column counts of the problem set
uint64_t problem_signature(int count, const hsrq_problem_t* probs) {
  Sig g;
  g.add((uint64_t)count);
  for (int p = 0; p < count; ++p) {
    g.add((uint64_t)probs[p].n);
    g.add((uint64_t)(probs[p].m > 0 ? count_cols(probs[p].m, probs[p].wi) : 0));
  }
  return g.v;
}

int heuristic_nb(int count, const hsrq_problem_t* probs) {
  int nmax = 0;
  for (int p = 0; p < count; ++p) nmax = std::max(nmax, probs[p].n);
  return nmax >= 2048 ? 128 : 64;
}

// options outside their documented values are rejected, never replaced by a
// default (the kernels exist for tile sizes 64 and 128 only)
bool opts_ok(const hsrq_opts_t* o) {
  if (!o) return true;
  if (o->nb != 0 && o->nb != 64 && o->nb != 128) return false;
  if (o->precision != 0 && o->precision != 1) return false;
  if (o->residual != 0 && o->residual != 1) return false;
  if (o->graph < -1 || o->graph > 1) return false;
  if (o->rotations != 0 && o->rotations != 1) return false;
  if (o->share_min_far < -1) return false;
  if (o->cols_per_block != 0 && o->cols_per_block != 32 && o->cols_per_block != 64) return false;
  if (o->cols_per_block == 32 && !(o->rotations == 1 && o->precision == 0)) return false;
  return true;
}

// tile size and far-block width: explicit options, else the autotuner's
// choice for this problem set, else a size rule (and 32 columns in the
// level-3 form: shorter far-tile blocks leave a shorter tail per step)
struct Tile {
  int nb, fcb;
};
bool l3_form(const hsrq_opts_t* o) { return o && o->rotations == 1 && o->precision == 0; }
Tile choose_tile(hsrq_handle_t h, int count, const hsrq_problem_t* probs, const hsrq_opts_t* o) {
  Tile t{heuristic_nb(count, probs), 32};
  if (h && !h->tuned.empty()) {
    const uint64_t key = problem_signature(count, probs);
    for (auto& e : h->tuned)
      if (e.key == key) t = Tile{e.nb, e.fcb};
  }
  if (o && (o->nb == 64 || o->nb == 128)) t.nb = o->nb;
  if (o && (o->cols_per_block == 32 || o->cols_per_block == 64)) t.fcb = o->cols_per_block;
  if (!l3_form(o)) t.fcb = 64;  // the one-at-a-time and FP32 far kernels take 64 columns
  return t;
}
int choose_nb(hsrq_handle_t h, int count, const hsrq_problem_t* probs, const hsrq_opts_t* o) {
  return choose_tile(h, count, probs, o).nb;
}

// pinned staging buffer created with the handle (grown by later calls that
// need more; the no-allocation entry point only uses what is there)
constexpr size_t kStagingBytes = size_t(2) << 20;

int ensure_staging(hsrq_handle_t h, size_t bytes) {
  if (h->staging_pending) {
    if (hipEventSynchronize(h->staging_ev) != hipSuccess) return HSRQ_ERR_HIP;
    h->staging_pending = false;
  }
  if (h->staging_bytes >= bytes) return HSRQ_OK;
  if (h->staging) hipHostFree(h->staging);
  h->staging = nullptr;
  h->staging_bytes = 0;
  size_t want = std::max<size_t>(bytes, kStagingBytes);
  if (hipHostMalloc(&h->staging, want, hipHostMallocDefault) != hipSuccess) {
    h->staging = nullptr;
    return HSRQ_ERR_ALLOC;
  }
  h->staging_bytes = want;
  return HSRQ_OK;
}

// Bracket one launch with profiling events when enabled.
// attach = true: the events go with a single kernel dispatch (start and end
// of that kernel, see launch_crit) instead of being recorded around it
struct ProfScope {
  hsrq_handle_t h;
  int kind;
  hipStream_t st;
  bool attach;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(hsrq_handle_t h_, int k, hipStream_t s_ = nullptr, bool attach_ = false)
      : h(h_), kind(k), st(s_ ? s_ : h_->stream), attach(attach_) {
    if (!h->prof) return;
    a = get();
    b = get();
    if (a && !attach) hipEventRecord(a, st);
  }
  ~ProfScope() {
    if (!h->prof || !a || !b) return;
    if (!attach) hipEventRecord(b, st);
    h->ev_used.push_back({kind, {a, b}});
  }
  hipEvent_t get() {
    if (!h->ev_pool.empty()) {
      hipEvent_t e = h->ev_pool.back();
      h->ev_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

// the handle's second stream and its three fork/join events, created with
// the handle (nothing is created inside a solve)
int create_sync(hsrq_handle_t h) {
  if (hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking) != hipSuccess) return HSRQ_ERR_HIP;
  for (hipEvent_t& e : h->sync_ev) {
    // ordering between the handle's two streams on one device: a release at
    // device scope is enough, and it spares the system-scope cache writeback
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming | hipEventDisableSystemFence) != hipSuccess)
      return HSRQ_ERR_HIP;
  }
  return HSRQ_OK;
}

// Enqueues the whole solve on stream s (and the handle's second stream for
// the far-tile kernels): head copy from the host image hb, then every kernel.
// do_output = false leaves the caller's X untouched (tuning, and the first
// pass of the mixed-precision solve); staging_ev, if given, is recorded right
// after the head copy.
int enqueue(hsrq_handle_t h, const Plan& P, int count, void* work, const void* hb, hipStream_t s, int do_resid,
            bool do_output, bool prof, hipEvent_t staging_ev) {
  if (hipMemcpyAsync(work, hb, P.head_bytes, hipMemcpyHostToDevice, s) != hipSuccess) return HSRQ_ERR_HIP;
  if (staging_ev && hipEventRecord(staging_ev, s) != hipSuccess) return HSRQ_ERR_HIP;
  if (P.blk_cols.empty()) return HSRQ_OK;
  const bool saved = h->prof;
  h->prof = prof;  // ProfScope reads the flag
  const ProbDesc* dd = at<ProbDesc>(work, P.o_desc);
  const Task* dt = at<Task>(work, P.o_tasks);
  const int T = (int)P.coff.size();
  hipStream_t a = h->aux;
  hipEvent_t ev_fork = h->sync_ev[0], ev_crit = h->sync_ev[1], ev_far = h->sync_ev[2];
  { ProfScope ps(h, HSRQ_K_PREP, s); launch_fill(at<double>(work, P.o_zero_all), (long long)P.zero_count, 0.0, s); }
  // the input scan on the second stream beside init (they share no data;
  // the scan needs the zeroed flags and norms, the first critical step the
  // scan's tile norms)
  hipEventRecord(ev_fork, s);
  hipStreamWaitEvent(a, ev_fork, 0);
  {
    ProfScope ps(h, HSRQ_K_PREP, a);
    launch_prep(dd, at<int4>(work, P.o_bprep), (int)P.blk_prep.size(), count, P.nmax, a);
  }
  { ProfScope ps(h, HSRQ_K_INIT, s); launch_init(dd, at<int4>(work, P.o_binit), (int)P.blk_init.size(), s); }
  hipEventRecord(ev_far, a);
  hipStreamWaitEvent(s, ev_far, 0);
  // steps: critical tasks on s, far tasks on the second stream; step t of
  // either kind waits for both kinds of step t-1.  (Letting the next
  // critical step start once only the far tile row next to the diagonal is
  // done was measured slower: the rest of the far tiles then hold the compute
  // units that the critical blocks, with their 83 KB of shared memory, need.)
  hipEventRecord(ev_fork, s);
  hipStreamWaitEvent(a, ev_fork, 0);
  for (int t = 0; t < T; ++t) {
    if (t > 0) {  // the records of step t-1
      hipStreamWaitEvent(s, ev_far, 0);
      hipStreamWaitEvent(a, ev_crit, 0);
    }
    if (P.ccnt[t] > 0) {
      ProfScope ps(h, HSRQ_K_CRIT, s, true);
      launch_crit(P.nb, P.prec, P.l3rot, share_step(P.fcnt[t], P.fcb, P.share) ? 1 : P.alone ? 2 : 0, dd, dt + P.coff[t],
                  P.ccnt[t], s, ps.a, ps.b);
    }
    if (P.fcnt[t] > 0) {
      if (t > 0) launch_gate(a);  // let the critical kernel reach the CUs first
      ProfScope ps(h, HSRQ_K_FAR, a, true);
      launch_far(P.nb, P.prec, P.l3rot, P.fcb, dd, dt + P.foff[t], P.fcnt[t], a, ps.a, ps.b);
    }
    hipEventRecord(ev_crit, s);
    hipEventRecord(ev_far, a);
  }
  // join: the second stream's last step (with no steps, its wait for the fork)
  if (T == 0) hipEventRecord(ev_far, a);
  hipStreamWaitEvent(s, ev_far, 0);
  {
    ProfScope ps(h, HSRQ_K_FINAL, s);
    launch_final(dd, at<int2>(work, P.o_bcols), (int)P.blk_cols.size(), at<int4>(work, P.o_bfin),
                 (int)P.blk_fin.size(), s);
  }
  if (do_resid == 1) {  // the FP64 residual of every shift
    ProfScope ps(h, HSRQ_K_RESID, s);
    launch_resid(dd, at<int4>(work, P.o_bout), (int)P.blk_out.size(), at<int2>(work, P.o_bcols),
                 (int)P.blk_cols.size(), s);
  } else if (do_resid == 2) {  // its sketched estimate (mixed precision's check)
    ProfScope ps(h, HSRQ_K_RESID, s);
    launch_sketch(dd, at<int2>(work, P.o_bskh), (int)P.blk_skh.size(), at<int4>(work, P.o_bout),
                  (int)P.blk_out.size(), at<int2>(work, P.o_bcols), (int)P.blk_cols.size(), s);
  }
  if (do_output) {
    ProfScope ps(h, HSRQ_K_OUTPUT, s);
    launch_output(dd, at<int4>(work, P.o_bout), (int)P.blk_out.size(), s);
  }
  h->prof = saved;
  if (hipGetLastError() != hipSuccess) return HSRQ_ERR_HIP;
  return HSRQ_OK;
}

// key of an instantiated launch sequence: everything the captured launches
// depend on (grid sizes, offsets into the workspace, the workspace itself);
// the descriptors and tables are re-copied from the staging image per replay
uint64_t plan_signature(const Plan& P, int count, void* work, bool want_res) {
  Sig g;
  g.add((uint64_t)P.nb);
  g.add((uint64_t)(P.prec * 2 + P.l3rot));
  g.add((uint64_t)(uint32_t)P.share);
  g.add((uint64_t)P.alone);
  g.add((uint64_t)P.fcb);
  g.add((uint64_t)count);
  g.add((uint64_t)reinterpret_cast<uintptr_t>(work));
  g.add((uint64_t)want_res);
  g.add((uint64_t)P.head_bytes);
  g.add((uint64_t)P.total_bytes);
  g.add((uint64_t)P.zero_count);
  g.add((uint64_t)P.o_zero_all);
  for (size_t v : {P.o_desc, P.o_tasks, P.o_bprep, P.o_bcols, P.o_binit, P.o_bout, P.o_bfin}) g.add(v);
  for (size_t v : {P.tasks.size(), P.blk_cols.size(), P.blk_prep.size(), P.blk_init.size(), P.blk_out.size(),
                   P.blk_fin.size(), P.coff.size()})
    g.add(v);
  for (size_t t = 0; t < P.coff.size(); ++t) {
    g.add((uint64_t)P.coff[t]);
    g.add((uint64_t)P.ccnt[t]);
    g.add((uint64_t)P.foff[t]);
    g.add((uint64_t)P.fcnt[t]);
  }
  return g.v;
}

void release_graph(hsrq_handle_s::GraphEntry& e) {
  for (auto& sl : e.slot) {
    if (sl.pending) hipEventSynchronize(sl.done);
    if (sl.exec) hipGraphExecDestroy(sl.exec);
    if (sl.staging) hipHostFree(sl.staging);
    if (sl.done) hipEventDestroy(sl.done);
    sl = hsrq_handle_s::GraphSlot();
  }
}

constexpr size_t kGraphCache = 8;

// Replays (capturing on first use) the launch sequence of plan P on stream s.
int run_graph(hsrq_handle_t h, const Plan& P, int count, const hsrq_problem_t* probs, void* work,
              const hsrq_opts_t* o, bool want_res, hipStream_t s) {
  const uint64_t key = plan_signature(P, count, work, want_res);
  hsrq_handle_s::GraphEntry* e = nullptr;
  for (auto& x : h->graphs)
    if (x.key == key) e = &x;
  if (!e) {
    if (h->graphs.size() >= kGraphCache) {  // evict the least recently used
      size_t lru = 0;
      for (size_t i = 1; i < h->graphs.size(); ++i)
        if (h->graphs[i].stamp < h->graphs[lru].stamp) lru = i;
      release_graph(h->graphs[lru]);
      h->graphs.erase(h->graphs.begin() + lru);
    }
    h->graphs.emplace_back();
    e = &h->graphs.back();
    e->key = key;
    e->head_bytes = P.head_bytes;
  }
  e->stamp = ++h->stamp;
  auto& sl = e->slot[e->next];
  e->next ^= 1;
  if (sl.pending) {
    if (hipEventSynchronize(sl.done) != hipSuccess) return HSRQ_ERR_HIP;
    sl.pending = false;
  }
  if (!sl.staging) {
    if (hipHostMalloc(&sl.staging, std::max<size_t>(P.head_bytes, 256), hipHostMallocDefault) != hipSuccess) {
      sl.staging = nullptr;
      return HSRQ_ERR_ALLOC;
    }
    if (hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) return HSRQ_ERR_HIP;
  }
  fill_staging(P, count, probs, work, o, static_cast<char*>(sl.staging));
  if (!sl.exec) {
    if (!h->cap && hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess) return HSRQ_ERR_HIP;
    if (hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return HSRQ_ERR_HIP;
    int st = enqueue(h, P, count, work, sl.staging, h->cap, want_res, true, false, nullptr);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(h->cap, &g);
    if (st == HSRQ_OK && (ec != hipSuccess || !g)) st = HSRQ_ERR_HIP;
    if (st == HSRQ_OK && hipGraphInstantiate(&sl.exec, g, nullptr, nullptr, 0) != hipSuccess) {
      sl.exec = nullptr;
      st = HSRQ_ERR_HIP;
    }
    if (g) hipGraphDestroy(g);
    if (st) return st;
  }
  if (hipGraphLaunch(sl.exec, s) != hipSuccess) return HSRQ_ERR_HIP;
  if (hipEventRecord(sl.done, s) != hipSuccess) return HSRQ_ERR_HIP;
  sl.pending = true;
  return HSRQ_OK;
}

bool wants_residual(const hsrq_opts_t* o, int count, const hsrq_problem_t* probs) {
  if (!(o && o->residual)) return false;
  for (int p = 0; p < count; ++p)
    if (!probs[p].resid) return false;
  return true;
}

// graph option: 1 = replay, -1 = eager launches, 0 = library default (replay
// for batched calls); profiling always launches eagerly
bool use_graph(hsrq_handle_t h, const hsrq_opts_t* o, bool batched) {
  if (h->prof) return false;
  const int g = o ? o->graph : 0;
  return g > 0 || (g == 0 && batched);
}

// The handle's pinned buffer of copy lists (read in place by the copy
// kernel), at least `need` bytes, once the kernels reading it have finished.
int ensure_lists(hsrq_handle_t h, size_t need) {
  if (h->lists_pending) {
    if (hipEventSynchronize(h->lists_ev) != hipSuccess) return HSRQ_ERR_HIP;
    h->lists_pending = false;
  }
  if (!h->lists_ev && hipEventCreateWithFlags(&h->lists_ev, hipEventDisableTiming) != hipSuccess)
    return HSRQ_ERR_HIP;
  if (h->lists_bytes < need) {
    if (h->lists) hipHostFree(h->lists);
    h->lists = nullptr;
    h->lists_bytes = 0;
    if (hipHostMalloc(&h->lists, need, hipHostMallocDefault) != hipSuccess) {
      h->lists = nullptr;
      return HSRQ_ERR_ALLOC;
    }
    h->lists_bytes = need;
  }
  return HSRQ_OK;
}

// Mixed precision (opts->precision == 1), in three phases:
//   1. the whole solve with FP32 tile-update products (every rotation, scale
//      factor, small solve and the normalisation stay FP64), and the FP64
//      residual ||H y - lambda y||_2 / (||H||_F ||y||_2) of every shift, with
//      the caller's X (the starting vectors) still untouched;
//   2. one synchronisation; a shift passes when its residual is at most
//      10 n eps (eps = 2^-52) and it converged;
//   3. the starting vectors of the failing shifts are gathered, solved again
//      all in FP64 (the fallback), and scattered back over the first pass's
//      results.  Shifts flagged singular or with invalid input are final.
// Workspace: [first pass | fallback pass | gathered columns | per-shift
// scalars], each region 256-byte aligned.
struct MixedLayout {
  size_t o_pass2 = 0, o_cols = 0, o_scal = 0, total = 0;
  std::vector<size_t> col_off, res_off;  // per problem, inside the regions
};

MixedLayout mixed_layout(int count, const hsrq_problem_t* probs, size_t pass_bytes) {
  MixedLayout L;
  size_t off = align_up(pass_bytes);
  L.o_pass2 = off;
  off = align_up(off + pass_bytes);
  L.o_cols = off;
  L.col_off.resize(count);
  for (int p = 0; p < count; ++p) {
    L.col_off[p] = off;
    const int nc = probs[p].m > 0 ? count_cols(probs[p].m, probs[p].wi) : 0;
    off = align_up(off + sizeof(double) * (size_t)probs[p].n * nc);
  }
  L.o_scal = off;
  L.res_off.resize(count);
  for (int p = 0; p < count; ++p) {
    L.res_off[p] = off;  // resid (m doubles), then E (m), info (m), mu (m) of the fallback
    off = align_up(off + (sizeof(double) * 2 + sizeof(int32_t) * 2) * (size_t)std::max(probs[p].m, 1) + 64);
  }
  L.total = off;
  return L;
}

int run_mixed(hsrq_handle_t h, int count, const hsrq_problem_t* probs, void* work, size_t work_bytes,
              const hsrq_opts_t* o) {
  h->last_fallback = 0;
  const int nb = choose_nb(h, count, probs, o);
  Plan P;
  build_plan(P, count, probs, nb);
  P.prec = 1;
  P.share = share_min(o);
  const MixedLayout L = mixed_layout(count, probs, P.total_bytes);
  if (!work || work_bytes < L.total || (reinterpret_cast<uintptr_t>(work) & (kAlign - 1)))
    return HSRQ_ERR_WORKSPACE;
  hipStream_t s = h->stream;
  int st = HSRQ_OK;
  // the check: the FP64 residual when the caller asks for residuals (it is
  // computed anyway), else its sketched estimate (O(8 n) per shift), which a
  // shift must meet with a factor 4 to spare
  bool want_full = false;
  for (int p = 0; p < count; ++p) want_full = want_full || probs[p].resid != nullptr;
  const double spare = want_full ? 1.0 : 0.25;
  // phase 1: residuals go to the caller's array if given, else to ours
  std::vector<hsrq_problem_t> q1(probs, probs + count);
  for (int p = 0; p < count; ++p)
    if (!q1[p].resid) q1[p].resid = at<double>(work, L.res_off[p]);
  if ((st = ensure_staging(h, P.head_bytes))) return st;
  hsrq_opts_t o1 = *o;
  fill_staging(P, count, q1.data(), work, &o1, static_cast<char*>(h->staging));
  st = enqueue(h, P, count, work, h->staging, s, want_full ? 1 : 2, false, h->prof, h->staging_ev);
  h->staging_pending = true;
  if (st) return st;
  // phase 2: the check
  std::vector<std::vector<int>> fail(count);
  size_t nfail = 0;
  {
    size_t mt = 0;
    std::vector<size_t> base(count);
    for (int p = 0; p < count; ++p) {
      base[p] = mt;
      mt += q1[p].m;
    }
    std::vector<double> res(std::max<size_t>(mt, 1));
    std::vector<int32_t> inf(std::max<size_t>(mt, 1));
    for (int p = 0; p < count; ++p) {
      const int m = q1[p].m;
      if (m == 0) continue;
      if (hipMemcpyAsync(res.data() + base[p], q1[p].resid, sizeof(double) * m, hipMemcpyDeviceToHost, s) !=
              hipSuccess ||
          hipMemcpyAsync(inf.data() + base[p], q1[p].info, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s) !=
              hipSuccess)
        return HSRQ_ERR_HIP;
    }
    if (hipStreamSynchronize(s) != hipSuccess) return HSRQ_ERR_HIP;
    for (int p = 0; p < count; ++p) {
      const double tol = 10.0 * q1[p].n * std::ldexp(1.0, -52) * spare;
      for (int l = 0; l < q1[p].m; ++l) {
        const int32_t in = inf[base[p] + l];
        const bool final_flag = in == 2 || in == 3 || in == 4;
        if (!final_flag && (in != 0 || !(res[base[p] + l] <= tol))) fail[p].push_back(l);
      }
      nfail += fail[p].size();
    }
  }
  if (nfail == 0) {
    ProfScope ps(h, HSRQ_K_OUTPUT, s);
    launch_output(at<ProbDesc>(work, P.o_desc), at<int4>(work, P.o_bout), (int)P.blk_out.size(), s);
    return hipGetLastError() == hipSuccess ? HSRQ_OK : HSRQ_ERR_HIP;
  }
  // phase 3: gather the starting vectors of the failing shifts (the caller's
  // X still holds them), then let the first pass write its output
  std::vector<hsrq_problem_t> q2;
  std::vector<int> src;                         // problem of each fallback problem
  std::vector<std::vector<double>> wr2, wi2;    // host shift lists of the fallback
  std::vector<std::vector<int>> col2;           // caller column of each gathered column
  std::vector<CopyEnt> gather, scatter;
  for (int p = 0; p < count; ++p) {
    if (fail[p].empty()) continue;
    const hsrq_problem_t& pr = probs[p];
    std::vector<int> firstcol(pr.m);
    for (int l = 0, c = 0; l < pr.m; ++l) {
      firstcol[l] = c;
      c += pr.wi[l] != 0.0 ? 2 : 1;
    }
    wr2.emplace_back();
    wi2.emplace_back();
    col2.emplace_back();
    double* G = at<double>(work, L.col_off[p]);
    int g = 0;
    for (int l : fail[p]) {
      wr2.back().push_back(pr.wr[l]);
      wi2.back().push_back(pr.wi[l]);
      const int w = pr.wi[l] != 0.0 ? 2 : 1;
      for (int k = 0; k < w; ++k) {
        col2.back().push_back(firstcol[l] + k);
        gather.push_back(CopyEnt{pr.X + (size_t)(firstcol[l] + k) * pr.ldx, G + (size_t)g * pr.n,
                                 (long long)sizeof(double) * pr.n});
        ++g;
      }
    }
    char* sc = at<char>(work, L.res_off[p]);
    const size_t mm = (size_t)std::max(pr.m, 1);
    hsrq_problem_t f{};
    f.n = pr.n;
    f.H = pr.H;
    f.ldh = pr.ldh;
    f.m = (int)fail[p].size();
    f.X = G;
    f.ldx = pr.n;
    f.resid = reinterpret_cast<double*>(sc);
    f.scale_exp = reinterpret_cast<int32_t*>(sc + sizeof(double) * mm);
    f.info = reinterpret_cast<int32_t*>(sc + (sizeof(double) + sizeof(int32_t)) * mm);
    f.scale_mant = reinterpret_cast<double*>(sc + (sizeof(double) + 2 * sizeof(int32_t)) * mm);
    q2.push_back(f);
    src.push_back(p);
  }
  for (size_t k = 0; k < q2.size(); ++k) {
    q2[k].wr = wr2[k].data();
    q2[k].wi = wi2[k].data();
  }
  // scatter list: the fallback's vectors and scalars over the first pass's
  for (size_t k = 0; k < q2.size(); ++k) {
    const hsrq_problem_t& pr = probs[src[k]];
    const hsrq_problem_t& f = q2[k];
    for (size_t g = 0; g < col2[k].size(); ++g)
      scatter.push_back(CopyEnt{f.X + g * (size_t)pr.n, pr.X + (size_t)col2[k][g] * pr.ldx,
                                (long long)sizeof(double) * pr.n});
    const std::vector<int>& fl = fail[src[k]];
    for (size_t j = 0; j < fl.size(); ++j) {
      const int l = fl[j];
      scatter.push_back(CopyEnt{f.scale_exp + j, pr.scale_exp + l, (long long)sizeof(int32_t)});
      scatter.push_back(CopyEnt{f.scale_mant + j, pr.scale_mant + l, (long long)sizeof(double)});
      scatter.push_back(CopyEnt{f.info + j, pr.info + l, (long long)sizeof(int32_t)});
      if (pr.resid) scatter.push_back(CopyEnt{f.resid + j, pr.resid + l, (long long)sizeof(double)});
    }
  }
  // both lists in one pinned buffer that the copy kernel reads in place
  {
    const size_t need = sizeof(CopyEnt) * (gather.size() + scatter.size());
    if ((st = ensure_lists(h, need))) return st;
    std::memcpy(h->lists, gather.data(), sizeof(CopyEnt) * gather.size());
    std::memcpy(static_cast<CopyEnt*>(h->lists) + gather.size(), scatter.data(), sizeof(CopyEnt) * scatter.size());
  }
  launch_copy(static_cast<const CopyEnt*>(h->lists), (int)gather.size(), s);
  {
    ProfScope ps(h, HSRQ_K_OUTPUT, s);
    launch_output(at<ProbDesc>(work, P.o_desc), at<int4>(work, P.o_bout), (int)P.blk_out.size(), s);
  }
  // the fallback, all FP64, in its own workspace region
  Plan P2;
  build_plan(P2, (int)q2.size(), q2.data(), nb);
  P2.prec = 0;
  P2.l3rot = o->rotations;
  P2.share = share_min(o);
  void* w2 = at<char>(work, L.o_pass2);
  if (P2.total_bytes > P.total_bytes) return HSRQ_ERR_WORKSPACE;
  if ((st = ensure_staging(h, P2.head_bytes))) return st;
  hsrq_opts_t o2 = *o;
  o2.precision = 0;
  fill_staging(P2, (int)q2.size(), q2.data(), w2, &o2, static_cast<char*>(h->staging));
  st = enqueue(h, P2, (int)q2.size(), w2, h->staging, s, want_full ? 1 : 0, true, h->prof, h->staging_ev);
  h->staging_pending = true;
  if (st) return st;
  launch_copy(static_cast<const CopyEnt*>(h->lists) + gather.size(), (int)scatter.size(), s);
  if (hipEventRecord(h->lists_ev, s) != hipSuccess) return HSRQ_ERR_HIP;
  h->lists_pending = true;
  h->last_fallback = nfail;
  return hipGetLastError() == hipSuccess ? HSRQ_OK : HSRQ_ERR_HIP;
}

int run(hsrq_handle_t h, int count, const hsrq_problem_t* probs, void* work, size_t work_bytes,
        const hsrq_opts_t* o, bool batched) {
  if (o && o->precision == 1) return run_mixed(h, count, probs, work, work_bytes, o);
  Plan P;
  const Tile tl = choose_tile(h, count, probs, o);
  build_plan(P, count, probs, tl.nb, tl.fcb);
  P.l3rot = o ? o->rotations : 0;
  P.share = share_min(o);
  if (!work || work_bytes < P.total_bytes || (reinterpret_cast<uintptr_t>(work) & (kAlign - 1)))
    return HSRQ_ERR_WORKSPACE;
  const bool want_res = wants_residual(o, count, probs);
  int st = HSRQ_OK;
  hipStream_t s = h->stream;
  if (use_graph(h, o, batched)) return run_graph(h, P, count, probs, work, o, want_res, s);
  st = ensure_staging(h, P.head_bytes);
  if (st) return st;
  fill_staging(P, count, probs, work, o, static_cast<char*>(h->staging));
  st = enqueue(h, P, count, work, h->staging, s, want_res, true, h->prof, h->staging_ev);
  h->staging_pending = true;
  return st;
}

}  // namespace

namespace hsrq {

int handle_device(hsrq_handle_t h) { return h->device; }
hipStream_t handle_stream(hsrq_handle_t h) { return h->stream; }
void* handle_blas(hsrq_handle_t h) {
  if (!h->blas && rocblas_create_handle(&h->blas) != rocblas_status_success) {
    h->blas = nullptr;
    return nullptr;
  }
  if (rocblas_set_stream(h->blas, h->stream) != rocblas_status_success) return nullptr;
  return h->blas;
}
bool opts_valid(const hsrq_opts_t* o) { return opts_ok(o); }

// The single-problem solve (precision 0) in the given workspace with nothing
// allocated or created: kernel-by-kernel launches on the handle's stream and
// its second stream, the plan staged through the handle's pinned buffer
// (created with the handle), no graph, no profiling events.
int run_noalloc(hsrq_handle_t h, const hsrq_problem_t& p, void* work, size_t work_bytes, const hsrq_opts_t* o) {
  Plan P;
  const Tile tl = choose_tile(h, 1, &p, o);
  build_plan(P, 1, &p, tl.nb, tl.fcb);
  P.l3rot = o ? o->rotations : 0;
  P.share = share_min(o);
  if (work_bytes < P.total_bytes || P.head_bytes > h->staging_bytes) return HSRQ_ERR_TOO_LARGE;
  if (h->staging_pending) {
    if (hipEventSynchronize(h->staging_ev) != hipSuccess) return HSRQ_ERR_HIP;
    h->staging_pending = false;
  }
  fill_staging(P, 1, &p, work, o, static_cast<char*>(h->staging));
  const int st = enqueue(h, P, 1, work, h->staging, h->stream, wants_residual(o, 1, &p), true, false,
                         h->staging_ev);
  h->staging_pending = true;
  return st;
}

}  // namespace hsrq

namespace {

// bytes of workspace for any tile size the library may pick (nb = 0)
size_t plan_bytes(hsrq_handle_t h, int count, const hsrq_problem_t* probs, const hsrq_opts_t* o) {
  size_t b = 0;
  const bool mixed = o && o->precision == 1;
  for (int nb : kNbCandidates) {
    if (o && (o->nb == 64 || o->nb == 128) && nb != o->nb) continue;
    for (int fcb : {32, 64}) {  // the task lists of 32-column far blocks are longer
      if (fcb == 32 && !l3_form(o)) continue;
      Plan P;
      build_plan(P, count, probs, nb, fcb);
      b = std::max(b, mixed ? mixed_layout(count, probs, P.total_bytes).total : P.total_bytes);
    }
  }
  (void)h;
  return b;
}

// ---------------------------------------------------------------------------
// Inverse iteration with restarts (Sec. 4.2, Algorithm 14) over groups of
// shifts sized by the workspace (Algorithm 15).
// ---------------------------------------------------------------------------
// The driver's workspace for a group of `cols` columns of order n: the
// solve's workspace (the plan's sizes depend on n and the column count only,
// so a problem of `cols` real shifts stands for any group of that many
// columns), the compacted columns of a restart, its per-shift outputs, and
// one column of zeros (the imaginary part of a complex shift's start).
struct InLayout {
  size_t solve = 0, o_cols = 0, o_scal = 0, o_zero = 0, total = 0;
};

InLayout in_layout(hsrq_handle_t h, int n, int cols, const hsrq_opts_t* o) {
  std::vector<double> z(std::max(cols, 1), 0.0);
  hsrq_problem_t p{};
  p.n = n;
  p.m = cols;
  p.wr = z.data();
  p.wi = z.data();
  InLayout L;
  L.solve = align_up(plan_bytes(h, 1, &p, o));
  size_t off = L.solve;
  L.o_cols = off;
  off = align_up(off + sizeof(double) * (size_t)n * cols);
  L.o_scal = off;  // resid, mu (doubles), then E, info (int32) of the restart's shifts
  off = align_up(off + (sizeof(double) * 2 + sizeof(int32_t) * 2) * (size_t)std::max(cols, 1) + 64);
  L.o_zero = off;
  off = align_up(off + sizeof(double) * (size_t)n);
  L.total = off;
  return L;
}

int run_hsrq3in(hsrq_handle_t h, int n, const double* H, int ldh, int m, const double* wr, const double* wi,
                const double* S, int lds, int ntries, double* X, int ldx, int32_t* E, double* mu, int32_t* info,
                int32_t* tries, double* resid, void* work, size_t work_bytes, const hsrq_opts_t* o) {
  if (!work || (reinterpret_cast<uintptr_t>(work) & (kAlign - 1))) return HSRQ_ERR_WORKSPACE;
  hipStream_t s = h->stream;
  std::vector<int> width(m), col(m);  // columns of each shift, first caller column
  int total = 0;
  bool any_cplx = false;
  for (int l = 0; l < m; ++l) {
    width[l] = wi[l] != 0.0 ? 2 : 1;
    any_cplx |= width[l] == 2;
    col[l] = total;
    total += width[l];
  }
  // group size (Algorithm 15): the most columns whose workspace fits
  int lo = 0, hi = total;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (in_layout(h, n, mid, o).total <= work_bytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int G = lo;
  if (G < 1 || (any_cplx && G < 2)) return HSRQ_ERR_WORKSPACE;
  const InLayout L = in_layout(h, n, G, o);
  double* zero = at<double>(work, L.o_zero);
  launch_fill(zero, n, 0.0, s);
  const bool want_res = resid && o && o->residual;
  int st = HSRQ_OK;
  for (int l0 = 0; l0 < m;) {
    int l1 = l0, cols = 0;
    while (l1 < m && cols + width[l1] <= G) cols += width[l1++];
    std::vector<int> act;  // shifts of the group not yet converged, in input order
    for (int l = l0; l < l1; ++l) act.push_back(l);
    for (int t = 0; t < ntries && !act.empty(); ++t) {
      const bool first = t == 0;
      const int ma = (int)act.size();
      std::vector<double> wr2(ma), wi2(ma);
      for (int k = 0; k < ma; ++k) {
        wr2[k] = wr[act[k]];
        wi2[k] = wi[act[k]];
      }
      // the first try solves in the caller's arrays (the group's columns are
      // contiguous there); a restart solves the remaining shifts compacted in
      // the workspace and copies its outputs back over the caller's
      hsrq_problem_t p{};
      p.n = n;
      p.H = H;
      p.ldh = ldh;
      p.m = ma;
      p.wr = wr2.data();
      p.wi = wi2.data();
      char* sc = at<char>(work, L.o_scal);
      if (first) {
        p.X = X + (size_t)col[l0] * ldx;
        p.ldx = ldx;
        p.scale_exp = E + l0;
        p.scale_mant = mu + l0;
        p.info = info + l0;
        p.resid = want_res ? resid + l0 : nullptr;
      } else {
        p.X = at<double>(work, L.o_cols);
        p.ldx = n;
        p.resid = want_res ? reinterpret_cast<double*>(sc) : nullptr;
        p.scale_mant = reinterpret_cast<double*>(sc) + G;
        p.scale_exp = reinterpret_cast<int32_t*>(reinterpret_cast<double*>(sc) + 2 * G);
        p.info = p.scale_exp + G;
      }
      // copy lists (pinned, read in place): the starting vector S(:, t) into
      // every column of the problem (zeros into the imaginary columns), then,
      // after the solve, a restart's outputs to the caller and the try index
      std::vector<CopyEnt> pre, post;
      for (int k = 0, c2 = 0; k < ma; ++k) {
        const int l = act[k];
        for (int q = 0; q < width[l]; ++q) {
          double* dst = p.X + (size_t)(c2 + q) * p.ldx;
          pre.push_back(CopyEnt{q == 0 ? S + (size_t)t * lds : zero, dst, (long long)sizeof(double) * n});
          if (!first) post.push_back(CopyEnt{dst, X + (size_t)(col[l] + q) * ldx, (long long)sizeof(double) * n});
        }
        c2 += width[l];
        if (!first) {
          post.push_back(CopyEnt{p.scale_exp + k, E + l, (long long)sizeof(int32_t)});
          post.push_back(CopyEnt{p.scale_mant + k, mu + l, (long long)sizeof(double)});
          post.push_back(CopyEnt{p.info + k, info + l, (long long)sizeof(int32_t)});
          if (want_res) post.push_back(CopyEnt{p.resid + k, resid + l, (long long)sizeof(double)});
        }
      }
      const size_t ents = pre.size() + post.size() + (tries ? ma : 0);
      if ((st = ensure_lists(h, sizeof(CopyEnt) * ents + sizeof(int32_t) * ma))) return st;
      CopyEnt* le = static_cast<CopyEnt*>(h->lists);
      int32_t* tv = reinterpret_cast<int32_t*>(le + ents);
      std::memcpy(le, pre.data(), sizeof(CopyEnt) * pre.size());
      std::memcpy(le + pre.size(), post.data(), sizeof(CopyEnt) * post.size());
      for (int k = 0; k < ma; ++k) {
        tv[k] = t;
        if (tries) le[pre.size() + post.size() + k] = CopyEnt{tv + k, tries + act[k], (long long)sizeof(int32_t)};
      }
      launch_copy(le, (int)pre.size(), s);
      if ((st = run(h, 1, &p, work, L.solve, o, false))) return st;
      launch_copy(le + pre.size(), (int)(ents - pre.size()), s);
      if (hipEventRecord(h->lists_ev, s) != hipSuccess) return HSRQ_ERR_HIP;
      h->lists_pending = true;
      // the flags decide the next try
      std::vector<int32_t> fl(ma);
      if (hipMemcpyAsync(fl.data(), p.info, sizeof(int32_t) * ma, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return HSRQ_ERR_HIP;
      std::vector<int> next;
      for (int k = 0; k < ma; ++k)
        if (fl[k] == 1) next.push_back(act[k]);
      act.swap(next);
    }
    l0 = l1;
  }
  return hipGetLastError() == hipSuccess ? HSRQ_OK : HSRQ_ERR_HIP;
}

}  // namespace

extern "C" {

int hsrq_hsrq3in_workspace_size(hsrq_handle_t h, int n, int m, const double* wi, const hsrq_opts_t* opts,
                                size_t* bytes) {
  if (!h) return -1;
  if (n < 1) return -2;
  if (m < 0) return -3;
  if (m > 0 && !wi) return -4;
  if (!opts_ok(opts) || (opts && opts->precision != 0)) return -5;
  if (!bytes) return -6;
  *bytes = in_layout(h, n, m > 0 ? count_cols(m, wi) : 1, opts).total;
  return HSRQ_OK;
}

int hsrq_hsrq3in(hsrq_handle_t h, int n, const double* H, int ldh, int m, const double* wr, const double* wi,
                 const double* S, int lds, int ntries, double* X, int ldx, int32_t* scale_exp,
                 double* scale_mant, int32_t* info, int32_t* tries, double* resid, void* work, size_t work_bytes,
                 const hsrq_opts_t* opts) {
  if (!h) return -1;
  if (n < 1) return -2;
  if (!H) return -3;
  if (ldh < n) return -4;
  if (m < 0) return -5;
  if (m > 0 && !wr) return -6;
  if (m > 0 && !wi) return -7;
  if (m > 0 && !S) return -8;
  if (lds < n) return -9;
  if (ntries < 1) return -10;
  if (m > 0 && !X) return -11;
  if (ldx < n) return -12;
  if (m > 0 && !scale_exp) return -13;
  if (m > 0 && !scale_mant) return -14;
  if (m > 0 && !info) return -15;
  if (!work) return -18;
  if (!opts_ok(opts) || (opts && opts->precision != 0)) return -20;
  if (m == 0) return HSRQ_OK;
  return run_hsrq3in(h, n, H, ldh, m, wr, wi, S, lds, ntries, X, ldx, scale_exp, scale_mant, info, tries, resid,
                     work, work_bytes, opts);
}

int hsrq_create(hsrq_handle_t* out, int device) {
  if (!out) return -1;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return HSRQ_ERR_HIP;
  if (crit_smem_init() != 0) return HSRQ_ERR_HIP;
  hsrq_handle_t h = new (std::nothrow) hsrq_handle_s();
  if (!h) return HSRQ_ERR_ALLOC;
  h->device = device;
  // everything a solve needs on the host side is created here: the staging
  // buffer, the second stream and its events, and the device's scratch
  // address for hsrq_dhsrq3_noalloc
  int st = HSRQ_OK;
  if (hipEventCreateWithFlags(&h->staging_ev, hipEventDisableTiming) != hipSuccess) st = HSRQ_ERR_HIP;
  if (st == HSRQ_OK) st = create_sync(h);
  if (st == HSRQ_OK) st = ensure_staging(h, kStagingBytes);
  if (st == HSRQ_OK && scratch_init(device) != 0) st = HSRQ_ERR_HIP;
  if (st) {
    hsrq_destroy(h);
    return st;
  }
  *out = h;
  return HSRQ_OK;
}

int hsrq_profile_enable(hsrq_handle_t h, int on) {
  if (!h) return -1;
  h->prof = on != 0;
  return HSRQ_OK;
}

int hsrq_fallback_count(hsrq_handle_t h, int64_t* count) {
  if (!h || !count) return -1;
  *count = (int64_t)h->last_fallback;
  return HSRQ_OK;
}

int hsrq_profile_read(hsrq_handle_t h, int nkinds, double* ms, int64_t* launches) {
  if (!h || nkinds < 0 || (nkinds > 0 && (!ms || !launches))) return -1;
  for (int k = 0; k < nkinds; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  int st = HSRQ_OK;
  for (auto& u : h->ev_used) {
    float t = 0.f;
    if (hipEventSynchronize(u.second.second) != hipSuccess ||
        hipEventElapsedTime(&t, u.second.first, u.second.second) != hipSuccess)
      st = HSRQ_ERR_HIP;
    if (u.first < nkinds) {
      ms[u.first] += t;
      launches[u.first] += 1;
    }
    h->ev_pool.push_back(u.second.first);
    h->ev_pool.push_back(u.second.second);
  }
  h->ev_used.clear();
  return st;
}

int hsrq_destroy(hsrq_handle_t h) {
  if (!h) return HSRQ_OK;
  if (h->staging_pending) hipEventSynchronize(h->staging_ev);
  for (auto& u : h->ev_used) {
    hipEventSynchronize(u.second.second);
    h->ev_pool.push_back(u.second.first);
    h->ev_pool.push_back(u.second.second);
  }
  for (auto& e : h->graphs) release_graph(e);
  h->graphs.clear();
  if (h->lists_pending) hipEventSynchronize(h->lists_ev);
  if (h->lists) hipHostFree(h->lists);
  if (h->lists_ev) hipEventDestroy(h->lists_ev);
  if (h->cap) hipStreamDestroy(h->cap);
  for (hipEvent_t e : h->ev_pool) hipEventDestroy(e);
  for (hipEvent_t e : h->sync_ev)
    if (e) hipEventDestroy(e);
  if (h->aux) {
    hipStreamSynchronize(h->aux);
    hipStreamDestroy(h->aux);
  }
  if (h->staging) hipHostFree(h->staging);
  if (h->staging_ev) hipEventDestroy(h->staging_ev);
  if (h->blas) rocblas_destroy_handle(h->blas);
  delete h;
  return HSRQ_OK;
}

int hsrq_set_stream(hsrq_handle_t h, void* stream) {
  if (!h) return -1;
  h->stream = static_cast<hipStream_t>(stream);
  return HSRQ_OK;
}

int hsrq_workspace_size_batched(hsrq_handle_t h, int count, const hsrq_problem_t* problems,
                                const hsrq_opts_t* opts, size_t* bytes) {
  if (!h || count < 0 || (count > 0 && !problems) || !bytes || !opts_ok(opts)) return HSRQ_ERR_ARG;
  for (int p = 0; p < count; ++p)
    if (problems[p].n < 1 || problems[p].m < 0 || (problems[p].m > 0 && !problems[p].wi)) return HSRQ_ERR_ARG;
  *bytes = plan_bytes(h, count, problems, opts);
  return HSRQ_OK;
}

int hsrq_workspace_size(hsrq_handle_t h, int n, int m, const double* wi, const hsrq_opts_t* opts,
                        size_t* bytes) {
  if (!h) return -1;
  if (n < 1) return -2;
  if (m < 0) return -3;
  if (m > 0 && !wi) return -4;
  if (!opts_ok(opts)) return -5;
  if (!bytes) return -6;
  std::vector<double> wr(m > 0 ? m : 1, 0.0);
  hsrq_problem_t p{};
  p.n = n; p.m = m; p.wr = wr.data(); p.wi = wi;
  *bytes = plan_bytes(h, 1, &p, opts);
  return HSRQ_OK;
}

int hsrq_dhsrq3(hsrq_handle_t h, int n, const double* H, int ldh, int m, const double* wr,
                const double* wi, double* X, int ldx, int32_t* scale_exp, double* scale_mant,
                int32_t* info, double* resid, void* work, size_t work_bytes, const hsrq_opts_t* opts) {
  if (!h) return -1;
  hsrq_problem_t p{n, H, ldh, m, wr, wi, X, ldx, scale_exp, scale_mant, info, resid};
  int st = check_problem(p);
  if (st) return st;
  if (!work) return -14;
  if (!opts_ok(opts)) return -16;
  if (m == 0) return HSRQ_OK;
  return run(h, 1, &p, work, work_bytes, opts, false);
}

int hsrq_dhsrq3_batched(hsrq_handle_t h, int count, const hsrq_problem_t* problems, void* work,
                        size_t work_bytes, const hsrq_opts_t* opts) {
  if (!h || count < 0 || (count > 0 && !problems) || !opts_ok(opts)) return HSRQ_ERR_ARG;
  for (int p = 0; p < count; ++p)
    if (check_problem(problems[p])) return HSRQ_ERR_ARG;
  if (count == 0) return HSRQ_OK;
  return run(h, count, problems, work, work_bytes, opts, true);
}

int hsrq_autotune(hsrq_handle_t h, int count, const hsrq_problem_t* problems, void* work, size_t work_bytes,
                  const hsrq_opts_t* opts, int* best_nb, int* best_cb, double* ms) {
  if (!h || count < 1 || !problems || !best_nb || !work || !opts_ok(opts)) return HSRQ_ERR_ARG;
  for (int p = 0; p < count; ++p)
    if (check_problem(problems[p])) return HSRQ_ERR_ARG;
  hsrq_opts_t o{};
  if (opts) o = *opts;
  o.graph = -1;
  const bool want_res = false;
  hipStream_t s = h->stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return HSRQ_ERR_HIP;
  Tile best{0, 0};
  double best_ms = 0.0;
  int st = HSRQ_OK;
  // the grid: tile sizes x far-block widths (32 only for the level-3 form);
  // ms[2 * (nb == 128) + (fcb == 64)]
  for (int c = 0; c < 4 && st == HSRQ_OK; ++c) {
    const int nb = kNbCandidates[c / 2], fcb = (c & 1) ? 64 : 32;
    if (ms) ms[c] = 0.0;
    if (fcb == 32 && !l3_form(&o)) continue;
    Plan P;
    build_plan(P, count, problems, nb, fcb);
    P.prec = o.precision == 1 ? 1 : 0;
    P.l3rot = o.rotations;
    P.share = share_min(&o);
    if (work_bytes < P.total_bytes || (reinterpret_cast<uintptr_t>(work) & (kAlign - 1))) continue;
    float t_best = 0.f;
    for (int rep = 0; rep < 3 && st == HSRQ_OK; ++rep) {  // first run warms up
      if ((st = ensure_staging(h, P.head_bytes))) break;
      fill_staging(P, count, problems, work, &o, static_cast<char*>(h->staging));
      if (hipEventRecord(e0, s) != hipSuccess) st = HSRQ_ERR_HIP;
      if (st == HSRQ_OK) st = enqueue(h, P, count, work, h->staging, s, want_res, false, false, h->staging_ev);
      h->staging_pending = true;
      if (st == HSRQ_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
        st = HSRQ_ERR_HIP;
      float t = 0.f;
      if (st == HSRQ_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) st = HSRQ_ERR_HIP;
      if (st == HSRQ_OK && rep > 0 && (rep == 1 || t < t_best)) t_best = t;
    }
    if (st) break;
    if (ms) ms[c] = t_best;
    if (best.nb == 0 || t_best < best_ms) {
      best = Tile{nb, fcb};
      best_ms = t_best;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st) return st;
  if (best.nb == 0) return HSRQ_ERR_WORKSPACE;
  const uint64_t key = problem_signature(count, problems);
  bool found = false;
  for (auto& e : h->tuned)
    if (e.key == key) {
      e.nb = best.nb;
      e.fcb = best.fcb;
      found = true;
    }
  if (!found) h->tuned.push_back(hsrq_handle_s::Tuned{key, best.nb, best.fcb});
  *best_nb = best.nb;
  if (best_cb) *best_cb = best.fcb;
  return HSRQ_OK;
}

int hsrq_debug_view(hsrq_handle_t h, int n, int m, const double* wi, const hsrq_opts_t* opts, void* work,
                    const double** C, const double** S, const double** PHI, const double** V, int* ld,
                    int* nb, int32_t* col_of) {
  if (!h || n < 1 || m < 0 || (m > 0 && !wi) || !work || !opts_ok(opts)) return HSRQ_ERR_ARG;
  std::vector<double> wr(m > 0 ? m : 1, 0.0);
  hsrq_problem_t p{};
  p.n = n; p.m = m; p.wr = wr.data(); p.wi = wi;
  Plan P;
  const Tile tl = choose_tile(h, 1, &p, opts);
  build_plan(P, 1, &p, tl.nb, tl.fcb);
  const ProbPlan& q = P.pp[0];
  if (C) *C = at<double>(work, q.o_C);
  if (S) *S = at<double>(work, q.o_S);
  if (PHI) *PHI = at<double>(work, q.o_PHI);
  if (V) *V = at<double>(work, q.o_V);
  if (ld) *ld = q.ld;
  if (nb) *nb = q.nb;
  if (col_of) {
    for (int c = 0; c < q.ncols; ++c)
      if (q.lay.coltype[c] != CT_CIM) col_of[q.lay.colshift[c]] = c;
  }
  return HSRQ_OK;
}

// Tuner cache: one line per problem-set signature, "<signature hex> <nb>
// <far-block width>", after a header line; entries loaded are merged into
// the handle's (a loaded entry replaces one with the same signature).
int hsrq_autotune_save(hsrq_handle_t h, const char* path) {
  if (!h || !path) return HSRQ_ERR_ARG;
  FILE* f = std::fopen(path, "w");
  if (!f) return HSRQ_ERR_ARG;
  bool ok = std::fprintf(f, "hsrq-tuner 2\n") > 0;
  for (auto& e : h->tuned)
    ok = ok && std::fprintf(f, "%016llx %d %d\n", (unsigned long long)e.key, e.nb, e.fcb) > 0;
  ok = (std::fclose(f) == 0) && ok;
  return ok ? HSRQ_OK : HSRQ_ERR_ARG;
}

int hsrq_autotune_load(hsrq_handle_t h, const char* path) {
  if (!h || !path) return HSRQ_ERR_ARG;
  FILE* f = std::fopen(path, "r");
  if (!f) return HSRQ_ERR_ARG;
  char head[32] = {0};
  int st = HSRQ_OK;
  if (!std::fgets(head, sizeof head, f) || std::strncmp(head, "hsrq-tuner 2", 12) != 0) st = HSRQ_ERR_ARG;
  std::vector<hsrq_handle_s::Tuned> got;
  unsigned long long key = 0;
  int nb = 0, fcb = 0;
  while (st == HSRQ_OK) {
    const int r = std::fscanf(f, "%llx %d %d", &key, &nb, &fcb);
    if (r == EOF) break;
    if (r != 3 || (nb != 64 && nb != 128) || (fcb != 32 && fcb != 64)) {
      st = HSRQ_ERR_ARG;
      break;
    }
    got.push_back(hsrq_handle_s::Tuned{(uint64_t)key, nb, fcb});
  }
  std::fclose(f);
  if (st) return st;  // nothing merged from a malformed file
  for (auto& g : got) {
    bool found = false;
    for (auto& e : h->tuned)
      if (e.key == g.key) {
        e = g;
        found = true;
      }
    if (!found) h->tuned.push_back(g);
  }
  return HSRQ_OK;
}

}  // extern "C"
